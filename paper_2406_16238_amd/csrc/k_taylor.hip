// One term of the Taylor series of the two-body exponential applied to the
// walker slabs (Sec. 2, eq. Bprop, exp(sqrt(dt) V_HS) phi by its series):
//   T_out = alpha * A_w T_in,   tacc += T_out   (acc = 1; acc = 0 leaves tacc
// alone, so T_in may be tacc itself; acc = 2 adds T_in + T_out, which folds in
// the term before),
// with A_w = sqrt(dt) V_HS of walker w held as real and imaginary M x M planes
// and T complex M x Nt, in three real products instead of four (the 3M form of
// a complex product): with A = Ar + i Ai and T = Tr + i Ti,
//   P1 = Ar Tr,  P2 = Ai Ti,  P3 = (Ar + Ai)(Tr + Ti),
//   A T = (P1 - P2) + i (P3 - P1 - P2),
// each an M x M by M x Nt real product, so a term costs 6 M^2 Nt flops instead
// of 8.  IMAG: A = i Ai (free projection, a real-field V_HS): A T = -Ai Ti +
// i Ai Tr, two products, and only the Ai plane is read.
//
// A workgroup owns BM = 4 TR NCW rows and all 16 TN >= Nt complex columns of
// one walker: compute wave w holds rows 4 TR w .. 4 TR (w + 1) - 1 and the
// three products of its rows, so the combination happens in registers and
// each lane writes whole complex entries.  The walker's A rows are read from
// memory once and its T (16 M Nt bytes) is shared by the M / BM row tiles,
// which the launch order places on one XCD.  Each wave issues TR x TN
// v_mfma_f64_4x4x4_4b_f64 per product and 4 contraction indices (lane
// 16k+4b+i supplies A_b[i][k], lane 16k+4b+j supplies B_b[k][j], lane
// 16i+4b+j receives D_b[i][j]; the four blocks are the four 4-column groups of
// one 16-column group, so A is the same for the four blocks).  M must be even
// and Nt at most 96; other shapes use the generic GEMM.
#include <type_traits>

#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

// The three-product term with both operands staged in LDS by DMA
// (buffer_load ... lds: lane L's 16 bytes land at the wave's LDS base + 16 L)
// through NBUF stages of TKC contraction indices.  One extra wave only copies:
// it issues the copies of chunk ch + NBUF - 1 while the NCW compute waves work
// on chunk ch, waits for chunk ch + 1, and meets them at the barrier that ends
// the chunk.  The compute waves issue no copies, so their LDS reads never wait
// on one (the compiler makes any LDS read of a wave with copies in flight wait
// for all of them).
// A stage holds the workgroup's rows of both V_HS planes ([plane][row][TKC],
// the 16-byte slots of row r swizzled by sw(r)) and TKC rows of T as they lie
// in memory (Nt interleaved complex entries a row).  In MFMA step s of a
// chunk, lane group g = lane >> 4 contracts index k0 + KS g + s
// (KS = TKC / 4), so a lane's A values of a chunk are consecutive in k and
// come in 16-byte reads.  Rows past M read row M - 1 (dropped at the store);
// contraction indices past M read zeros or finite values of the same walker
// against T rows that are zero: the copies' buffer resources end at the
// walker's data, and a buffer load whose offset (the VGPR part, which carries
// the whole offset here) lies past the end returns zero.
__device__ __forceinline__ __amdgpu_buffer_rsrc_t buffer_rsrc(const void *base, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), (short)0, (int)bytes, 0x00020000);
}
// one 16-byte LDS copy per lane (non-template: the host pass drops a kernel
// template that names this builtin itself)
__device__ __forceinline__ void lds_copy16(__amdgpu_buffer_rsrc_t r, void *lds, int voff) {
  __builtin_amdgcn_raw_ptr_buffer_load_lds(r, (__attribute__((address_space(3))) void *)lds, 16, voff, 0, 0, 0);
}

template <int TR, int TN, bool IMAG, int TKC_, int NBUF, int NCW>
__global__ __launch_bounds__(64 * (NCW + 1)) __attribute__((amdgpu_waves_per_eu(3))) void k_taylor3s(const double *__restrict__ vhs,
                                                                 const double2 *__restrict__ tin,
                                                                 double2 *__restrict__ tout,
                                                                 double2 *__restrict__ tacc, int M, int Nt, int W,
                                                                 int nrt, double alpha, int acc) {
  constexpr int BM = 4 * TR * NCW, KS = TKC_ / 4, SLOTS = TKC_ / 2;   // 16-byte slots per staged A row
  constexpr int NPL = IMAG ? 1 : 2;
  constexpr int AROWS = NPL * BM, AI = (AROWS * SLOTS + 63) / 64;    // copy instructions of an A stage
  constexpr int TI = (TKC_ * 16 * TN + 63) / 64;                    // of a T stage (Nt <= 16 TN entries a row)
  constexpr int NI = AI + TI, D = NBUF - 1;                         // D chunks in flight
  static_assert((D - 1) * NI < 64, "vmcnt range");
  static_assert(NCW % 4 == 0, "compute waves spread evenly over the SIMDs");
  auto sw = [](int r) { return TKC_ == 16 ? (r >> 1) & 1 : 0; };
  extern __shared__ __attribute__((aligned(16))) double2 ssh[];
  double2 *sA = ssh;                                               // [NBUF][AI * 64]
  double2 *sT = ssh + NBUF * AI * 64;                              // [NBUF][TI * 64]

  const int ntiles = W * nrt;
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int t = x * per + min(x, rem) + jx;
  const int w = t / nrt, i0 = (t - w * nrt) * BM;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wm = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nchunk = (M + TKC_ - 1) / TKC_;
  const int rbase = i0 + wm * 4 * TR;
  const bool live = rbase < M;   // a compute wave whose rows all lie past M issues no MFMA

  if (wm == NCW) {
    // the copy wave: instruction q of a stage is A block q (q < AI) or T block
    // q - AI; the lane's byte offset at chunk 0 (a chunk adds k0 * 8 for A,
    // k0 * Nt * 16 for T)
    const int MM = M * M;
    const __amdgpu_buffer_rsrc_t ares =
        buffer_rsrc(vhs + (size_t)w * 2 * MM + (IMAG ? MM : 0), (uint32_t)NPL * MM * 8u);
    const __amdgpu_buffer_rsrc_t tres = buffer_rsrc(tin + (size_t)w * M * Nt, (uint32_t)M * Nt * 16u);
    int qoff[NI];
#pragma unroll
    for (int q = 0; q < NI; ++q) {
      if (q < AI) {
        const int e = q * 64 + lane, row = e / SLOTS, slot = e - row * SLOTS;
        const int p = row / BM, r = row - p * BM;
        qoff[q] = (p * MM + min(i0 + r, M - 1) * M + 2 * (slot ^ sw(r))) * 8;
      } else {
        qoff[q] = ((q - AI) * 64 + lane) * 16;
      }
    }
    auto issue = [&](int ch) {
      const int buf = ch % NBUF, k0 = ch * TKC_;
#pragma unroll
      for (int q = 0; q < NI; ++q) {
        if (q < AI)
          lds_copy16(ares, sA + (buf * AI + q) * 64, qoff[q] + k0 * 8);
        else
          lds_copy16(tres, sT + (buf * TI + q - AI) * 64, qoff[q] + k0 * Nt * 16);
      }
    };
#pragma unroll
    for (int c = 0; c < D; ++c) issue(c);
    // the copies complete in order: with those of the D - 1 later chunks at
    // most outstanding, the next chunk has landed.  Copies past the last chunk
    // read zeros or unused values into stages no one reads, which keeps every
    // wait's count the same.  Bare barriers: a fence would wait for every copy.
    AFQMC_WAIT_VMCNT((D - 1) * NI);
    __builtin_amdgcn_s_barrier();
    for (int c = 0; c < nchunk; ++c) {
      issue(c + D);
      AFQMC_WAIT_VMCNT((D - 1) * NI);
      __builtin_amdgcn_s_barrier();
    }
    AFQMC_WAIT_VMCNT(0);   // no copy may outlive the workgroup's LDS
    return;
  }

  const int lr = lane & 15, lk = lane >> 4, l4 = lane & 3;
  double p1[TR][TN], p2[TR][TN], p3[TR][TN];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) p1[i][j] = p2[i][j] = p3[i][j] = 0.0;

  // operands of one MFMA step: the lane's A pair of steps 2h, 2h + 1 (slab i,
  // plane p) and its B entries (Re, Im); those of the next step are read
  // before the MFMAs of this one.
  auto read_a = [&](int stage, int h, double2 (&dst)[NPL][TR]) {
    const double2 *a = sA + stage * AI * 64;
#pragma unroll
    for (int p = 0; p < NPL; ++p)
#pragma unroll
      for (int i = 0; i < TR; ++i) {
        const int r = wm * 4 * TR + 4 * i + l4;
        dst[p][i] = a[(p * BM + r) * SLOTS + (((KS / 2) * lk + h) ^ sw(r))];
      }
  };
  auto read_b = [&](int stage, int s, double2 (&dst)[TN]) {
    const double2 *b = sT + stage * TI * 64 + (KS * lk + s) * Nt + lr;
#pragma unroll
    for (int j = 0; j < TN; ++j) dst[j] = b[16 * j];
  };
  double2 av[NPL][TR], bv[TN];
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    if (!live) {
      __syncthreads();
      continue;
    }
    const int stage = ch % NBUF;
    read_a(stage, 0, av);
    read_b(stage, 0, bv);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      double2 an[NPL][TR], bn[TN];
      const bool last = s + 1 == KS;
      if (!last) {
        read_b(stage, s + 1, bn);
        if ((s + 1) % 2 == 0) read_a(stage, (s + 1) / 2, an);
      }
      double yr[TN], yi[TN];
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        yr[j] = bv[j].x;
        yi[j] = bv[j].y;
      }
      auto aval = [&](int p, int i) { return (s & 1) ? av[p][i].y : av[p][i].x; };
      if constexpr (IMAG) {
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          const double xi = aval(0, i);
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi, yr[j], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi, yi[j], p2[i][j], 0, 0, 0);
          }
        }
      } else {
        double xr[TR], xi[TR];
#pragma unroll
        for (int i = 0; i < TR; ++i) {
          xr[i] = aval(0, i);
          xi[i] = aval(1, i);
        }
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xr[i], yr[j], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi[i], yi[j], p2[i][j], 0, 0, 0);
          }
#pragma unroll
        for (int i = 0; i < TR; ++i) xr[i] += xi[i];
#pragma unroll
        for (int j = 0; j < TN; ++j) yr[j] += yi[j];
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j)
            p3[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xr[i], yr[j], p3[i][j], 0, 0, 0);
      }
      if (!last) {
#pragma unroll
        for (int j = 0; j < TN; ++j) bv[j] = bn[j];
        if ((s + 1) % 2 == 0)
#pragma unroll
          for (int p = 0; p < NPL; ++p)
#pragma unroll
            for (int i = 0; i < TR; ++i) av[p][i] = an[p][i];
      }
    }
    __syncthreads();
  }
  if (!live) return;

  double2 *to = tout + (size_t)w * M * Nt;
  double2 *ta = tacc + (size_t)w * M * Nt;
  const double2 *tw = tin + (size_t)w * M * Nt;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int gi = rbase + 4 * i + lk;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = 16 * j + lr;
      if (gi < M && c < Nt) {
        const size_t off = (size_t)gi * Nt + c;
        const double re = IMAG ? -p2[i][j] : p1[i][j] - p2[i][j];
        const double im = IMAG ? p1[i][j] : (p3[i][j] - p1[i][j]) - p2[i][j];
        const double2 v = make_double2(alpha * re, alpha * im);
        to[off] = v;
        if (acc) {
          const double2 o = ta[off];
          double2 u = v;
          if (acc == 2) {
            const double2 x = tw[off];
            u = make_double2(x.x + v.x, x.y + v.y);
          }
          ta[off] = make_double2(o.x + u.x, o.y + u.y);
        }
      }
    }
  }
}

// The same term without a copy wave, for three or four workgroups per CU: each of the
// NCW waves issues its share of every stage's copies (instructions q = wave +
// NCW n) at the top of a chunk, NBUF - 1 chunks ahead, waits for its share of
// the next chunk and meets the others at a bare barrier.  Its LDS reads go
// through native vector types, which the compiler does not make wait for the
// wave's own copies in flight.
typedef double v2d __attribute__((ext_vector_type(2)));
__device__ __forceinline__ void bare_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

template <int TR, int TN, bool IMAG, int TKC_, int NBUF, int NCW, int OCC>
__global__ __launch_bounds__(64 * NCW, OCC) void k_taylor3w(const double *__restrict__ vhs,
                                                             const double2 *__restrict__ tin,
                                                             double2 *__restrict__ tout,
                                                             double2 *__restrict__ tacc, int M, int Nt, int W,
                                                             int nrt, double alpha, int acc) {
  constexpr int BM = 4 * TR * NCW, KS = TKC_ / 4, SLOTS = TKC_ / 2;
  constexpr int NPL = IMAG ? 1 : 2;
  constexpr int AROWS = NPL * BM, AI = (AROWS * SLOTS + 63) / 64;
  constexpr int TI = (TKC_ * 16 * TN + 63) / 64;
  constexpr int NI = AI + TI, D = NBUF - 1;
  constexpr int NQ = (NI + NCW - 1) / NCW, CMIN = NI / NCW;   // copies per wave and stage: at most, at least
  static_assert((D - 1) * NQ < 64, "vmcnt range");
  auto sw = [](int r) { return TKC_ == 16 ? (r >> 1) & 1 : 0; };
  extern __shared__ __attribute__((aligned(16))) double2 ssh[];
  double2 *sA = ssh;
  double2 *sT = ssh + NBUF * AI * 64;

  const int ntiles = W * nrt;
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int t = x * per + min(x, rem) + jx;
  const int w = t / nrt, i0 = (t - w * nrt) * BM;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wm = __builtin_amdgcn_readfirstlane(tid >> 6);
  const int nchunk = (M + TKC_ - 1) / TKC_;
  const int rbase = i0 + wm * 4 * TR;
  const bool live = rbase < M;

  const int MM = M * M;
  const __amdgpu_buffer_rsrc_t ares = buffer_rsrc(vhs + (size_t)w * 2 * MM + (IMAG ? MM : 0), (uint32_t)NPL * MM * 8u);
  const __amdgpu_buffer_rsrc_t tres = buffer_rsrc(tin + (size_t)w * M * Nt, (uint32_t)M * Nt * 16u);
  int qoff[NQ];
#pragma unroll
  for (int n = 0; n < NQ; ++n) {
    const int q = wm + NCW * n;
    int off;
    if (q < AI) {
      const int e = q * 64 + lane, row = e / SLOTS, slot = e - row * SLOTS;
      const int p = row / BM, r = row - p * BM;
      off = (p * MM + min(i0 + r, M - 1) * M + 2 * (slot ^ sw(r))) * 8;
    } else {
      off = ((q - AI) * 64 + lane) * 16;
    }
    qoff[n] = off;
  }
  auto issue = [&](int ch) {
    const int buf = ch % NBUF, k0 = ch * TKC_;
#pragma unroll
    for (int n = 0; n < NQ; ++n) {
      const int q = wm + NCW * n;
      if (NI % NCW != 0 && q >= NI) break;   // uniform in the wave
      if (q < AI)
        lds_copy16(ares, sA + (buf * AI + q) * 64, qoff[n] + k0 * 8);
      else
        lds_copy16(tres, sT + (buf * TI + q - AI) * 64, qoff[n] + k0 * Nt * 16);
    }
  };

  const int lr = lane & 15, lk = lane >> 4, l4 = lane & 3;
  double p1[TR][TN], p2[TR][TN], p3[TR][TN];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) p1[i][j] = p2[i][j] = p3[i][j] = 0.0;
  auto read_a = [&](int stage, int h, v2d (&dst)[NPL][TR]) {
    const v2d *a = reinterpret_cast<const v2d *>(sA + stage * AI * 64);
#pragma unroll
    for (int p = 0; p < NPL; ++p)
#pragma unroll
      for (int i = 0; i < TR; ++i) {
        const int r = wm * 4 * TR + 4 * i + l4;
        dst[p][i] = a[(p * BM + r) * SLOTS + (((KS / 2) * lk + h) ^ sw(r))];
      }
  };
  auto read_b = [&](int stage, int s, v2d (&dst)[TN]) {
    const v2d *b = reinterpret_cast<const v2d *>(sT + stage * TI * 64 + (KS * lk + s) * Nt + lr);
#pragma unroll
    for (int j = 0; j < TN; ++j) dst[j] = b[16 * j];
  };

  // chunks 0 .. D-1 in flight; copies past the last chunk read zeros or unused
  // values into stages no one reads, which keeps every wait's count the same
#pragma unroll
  for (int c = 0; c < D; ++c) issue(c);
  AFQMC_WAIT_VMCNT((D - 1) * CMIN);   // this wave's copies of chunk 0 (a wave with more waits a little longer)
  bare_barrier();
  v2d av[NPL][TR], bv[TN];
  for (int ch = 0; ch < nchunk; ++ch) {
    issue(ch + D);   // into the stage read in chunk ch - 1
    if (live) {
      const int stage = ch % NBUF;
      read_a(stage, 0, av);
      read_b(stage, 0, bv);
#pragma unroll
      for (int s = 0; s < KS; ++s) {
        v2d an[NPL][TR], bn[TN];
        const bool last = s + 1 == KS;
        if (!last) {
          read_b(stage, s + 1, bn);
          if ((s + 1) % 2 == 0) read_a(stage, (s + 1) / 2, an);
        }
        double yr[TN], yi[TN];
#pragma unroll
        for (int j = 0; j < TN; ++j) {
          yr[j] = bv[j].x;
          yi[j] = bv[j].y;
        }
        auto aval = [&](int p, int i) { return (s & 1) ? av[p][i].y : av[p][i].x; };
        if constexpr (IMAG) {
#pragma unroll
          for (int i = 0; i < TR; ++i) {
            const double xi = aval(0, i);
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi, yr[j], p1[i][j], 0, 0, 0);
              p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi, yi[j], p2[i][j], 0, 0, 0);
            }
          }
        } else {
          double xr[TR], xi[TR];
#pragma unroll
          for (int i = 0; i < TR; ++i) {
            xr[i] = aval(0, i);
            xi[i] = aval(1, i);
          }
#pragma unroll
          for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j) {
              p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xr[i], yr[j], p1[i][j], 0, 0, 0);
              p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi[i], yi[j], p2[i][j], 0, 0, 0);
            }
#pragma unroll
          for (int i = 0; i < TR; ++i) xr[i] += xi[i];
#pragma unroll
          for (int j = 0; j < TN; ++j) yr[j] += yi[j];
#pragma unroll
          for (int i = 0; i < TR; ++i)
#pragma unroll
            for (int j = 0; j < TN; ++j)
              p3[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xr[i], yr[j], p3[i][j], 0, 0, 0);
        }
        if (!last) {
#pragma unroll
          for (int j = 0; j < TN; ++j) bv[j] = bn[j];
          if ((s + 1) % 2 == 0)
#pragma unroll
            for (int p = 0; p < NPL; ++p)
#pragma unroll
              for (int i = 0; i < TR; ++i) av[p][i] = an[p][i];
        }
      }
    }
    __builtin_amdgcn_sched_barrier(0);
    AFQMC_WAIT_VMCNT((D - 1) * CMIN);   // this wave's copies of chunk ch + 1
    bare_barrier();
  }
  AFQMC_WAIT_VMCNT(0);   // no copy may outlive the workgroup's LDS
  if (!live) return;

  double2 *to = tout + (size_t)w * M * Nt;
  double2 *ta = tacc + (size_t)w * M * Nt;
  const double2 *tw = tin + (size_t)w * M * Nt;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int gi = rbase + 4 * i + lk;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = 16 * j + lr;
      if (gi < M && c < Nt) {
        const size_t off = (size_t)gi * Nt + c;
        const double re = IMAG ? -p2[i][j] : p1[i][j] - p2[i][j];
        const double im = IMAG ? p1[i][j] : (p3[i][j] - p1[i][j]) - p2[i][j];
        const double2 v = make_double2(alpha * re, alpha * im);
        to[off] = v;
        if (acc) {
          const double2 o = ta[off];
          double2 u = v;
          if (acc == 2) {
            const double2 x = tw[off];
            u = make_double2(x.x + v.x, x.y + v.y);
          }
          ta[off] = make_double2(o.x + u.x, o.y + u.y);
        }
      }
    }
  }
}

namespace {
constexpr int kTaylorKc = 8;     // contraction indices per stage
constexpr int kTaylorStages = 4;

template <int TR, int NCW, int TN, bool IMAG>
hipError_t run_taylor3s(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st,
                        int w0, int acc) {
  constexpr int BM = 4 * TR * NCW, TK = kTaylorKc, NB = kTaylorStages;
  const int ai = ((IMAG ? 1 : 2) * BM * (TK / 2) + 63) / 64, ti = (TK * 16 * TN + 63) / 64;
  const size_t lds = (size_t)NB * (ai + ti) * 64 * sizeof(double2);
  auto k = k_taylor3s<TR, TN, IMAG, TK, NB, NCW>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       80 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 80 * 1024) return hipErrorInvalidValue;
  const int nrt = (s.M + BM - 1) / BM;
  const size_t wt = (size_t)w0 * s.M * s.Nt;
  hipLaunchKernelGGL(k, dim3((unsigned)(W * nrt)), dim3(64 * (NCW + 1)), lds, st, s.vhs + (size_t)w0 * 2 * s.M * s.M,
                     tin + wt, tout + wt, s.tacc + wt, s.M, s.Nt, W, nrt, alpha, acc);
  return hipGetLastError();
}

template <int TR, bool IMAG>
hipError_t run_taylor3s_tn(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st,
                           int w0, int acc) {
  switch ((s.Nt + 15) / 16) {
    case 1: return run_taylor3s<TR, 4, 1, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
    case 2: return run_taylor3s<TR, 4, 2, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
    case 3: return run_taylor3s<TR, 4, 3, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
    case 4: return run_taylor3s<TR, 4, 4, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
    case 5: return run_taylor3s<TR, 4, 5, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
    // 96 columns: 32-row tiles keep the three accumulator sets in registers
    default: return run_taylor3s<2, 4, 6, IMAG>(s, tin, tout, alpha, W, st, w0, acc);
  }
}
// NB stages, OCC workgroups per CU (LDS and registers permitting)
template <int TR, int TN, bool IMAG, int NB, int OCC>
hipError_t run_taylor3w(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st,
                        int w0, int acc) {
  constexpr int NCW = 4, BM = 4 * TR * NCW, TK = kTaylorKc;
  const int ai = ((IMAG ? 1 : 2) * BM * (TK / 2) + 63) / 64, ti = (TK * 16 * TN + 63) / 64;
  const size_t lds = (size_t)NB * (ai + ti) * 64 * sizeof(double2);
  auto k = k_taylor3w<TR, TN, IMAG, TK, NB, NCW, OCC>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       80 * 1024);
    if (e != hipSuccess) return e;
    attr = true;
  }
  if (lds > 80 * 1024) return hipErrorInvalidValue;
  const int nrt = (s.M + BM - 1) / BM;
  const size_t wt = (size_t)w0 * s.M * s.Nt;
  hipLaunchKernelGGL(k, dim3((unsigned)(W * nrt)), dim3(64 * NCW), lds, st, s.vhs + (size_t)w0 * 2 * s.M * s.M,
                     tin + wt, tout + wt, s.tacc + wt, s.M, s.Nt, W, nrt, alpha, acc);
  return hipGetLastError();
}

// 48-row tiles: three stages (48 KB), three workgroups per CU; 32-row tiles:
// two stages (28 KB), four workgroups per CU (measured faster than three
// stages at three: more workgroups cover one's barrier wait better than a
// deeper pipeline); 96 columns: 32-row tiles, three stages at three
template <int TR, bool IMAG>
hipError_t run_taylor3w_tn(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st,
                           int w0, int acc) {
  constexpr int NB = TR == 2 ? 2 : 3, OCC = TR == 2 ? 4 : 3;
  switch ((s.Nt + 15) / 16) {
    case 1: return run_taylor3w<TR, 1, IMAG, NB, OCC>(s, tin, tout, alpha, W, st, w0, acc);
    case 2: return run_taylor3w<TR, 2, IMAG, NB, OCC>(s, tin, tout, alpha, W, st, w0, acc);
    case 3: return run_taylor3w<TR, 3, IMAG, NB, OCC>(s, tin, tout, alpha, W, st, w0, acc);
    case 4: return run_taylor3w<TR, 4, IMAG, NB, OCC>(s, tin, tout, alpha, W, st, w0, acc);
    case 5: return run_taylor3w<TR, 5, IMAG, NB, OCC>(s, tin, tout, alpha, W, st, w0, acc);
    default: return run_taylor3w<2, 6, IMAG, 3, 3>(s, tin, tout, alpha, W, st, w0, acc);
  }
}
}  // namespace

bool taylor_mfma_supported(int M, int Nt) { return M % 2 == 0 && Nt >= 1 && Nt <= 96; }

bool taylor_walker_split(const System &s) {
  return s.use_mfma_gemm && s.taylor_kernel && taylor_mfma_supported(s.M, s.Nt);
}

int taylor_shapes(const System &s) { return s.prop32 ? 3 : 4; }

// shape 0: 48-row tiles, 1: 32-row tiles (copy wave, two workgroups per CU);
// 2: 48-row tiles, 3: 32-row tiles (no copy wave; three and four workgroups per CU)
hipError_t launch_taylor_mfma(const System &s, const double2 *tin, double2 *tout, double alpha, int W,
                              hipStream_t st, int kbeg, int w0, int acc) {
  const bool imag = kbeg != 0;
  if (imag && kbeg != s.M) return hipErrorInvalidValue;
  if (s.taylor_shape == 2)
    return imag ? run_taylor3w_tn<3, true>(s, tin, tout, alpha, W, st, w0, acc)
                : run_taylor3w_tn<3, false>(s, tin, tout, alpha, W, st, w0, acc);
  if (s.taylor_shape == 3)
    return imag ? run_taylor3w_tn<2, true>(s, tin, tout, alpha, W, st, w0, acc)
                : run_taylor3w_tn<2, false>(s, tin, tout, alpha, W, st, w0, acc);
  if (s.taylor_shape == 1)
    return imag ? run_taylor3s_tn<2, true>(s, tin, tout, alpha, W, st, w0, acc)
                : run_taylor3s_tn<2, false>(s, tin, tout, alpha, W, st, w0, acc);
  return imag ? run_taylor3s_tn<3, true>(s, tin, tout, alpha, W, st, w0, acc)
              : run_taylor3s_tn<3, false>(s, tin, tout, alpha, W, st, w0, acc);
}

}  // namespace afqmc
