// Exchange energy of the local energy (Sec. 2, eq. Eloc, by Wick's theorem with
// the Cholesky integrals):
//   EK = -1/2 sum_g sum_s Tr(T^{g s} T^{g s}),  T^{g s} = Ltilde^{g s} Theta_s,
// with Ltilde^{g s} = Psi_s^T L^g (N_s x M) and Theta_s (M x N_s) complex.
// T is never written to HBM: each workgroup forms T for a block of Cholesky
// vectors of one (walker, spin) in registers, transposes it through LDS for
// the trace, and writes one complex partial sum.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int EXK = 32;  // contraction rows staged per LDS pass

size_t exchange_lds_bytes(int np, int gb) {
  const size_t stage = (size_t)gb * EXK * np * sizeof(double) + (size_t)EXK * np * sizeof(double2);
  const size_t epi = (size_t)gb * np * np * sizeof(double2);
  return stage > epi ? stage : epi;
}
}  // namespace

void exchange_geometry(int nmax, int *gb, size_t *lds) {
  const int np = ((nmax + 3) / 4) * 4;
  const int groups = (np / 4) * (np / 4);
  int g = kThreads / groups;
  if (g > 16) g = 16;
  if (g < 1) g = 1;
  while (g > 1 && exchange_lds_bytes(np, g) > 64512) --g;  // leave room for static LDS
  *gb = g;
  *lds = exchange_lds_bytes(np, g);
}

// grid (ngb, 2, W); block kThreads.  Thread t owns a 4x4 block (ig, jg) of T for
// Cholesky vector g0 + t / groups.
__global__ __launch_bounds__(kThreads) void k_exchange_v1(const double *__restrict__ LtT,
                                                         const double2 *__restrict__ theta, int M, int Na,
                                                         int Nb, int G, int GB, int ngb,
                                                         double2 *__restrict__ ekpart) {
  extern __shared__ double smem[];
  __shared__ double red[4 * 2];
  const int gb = blockIdx.x, s = blockIdx.y, w = blockIdx.z, tid = threadIdx.x;
  const int N = s ? Nb : Na, off = s ? Na : 0, Nt = Na + Nb;
  const int NP = ((N + 3) / 4) * 4, NG4 = NP > 0 ? NP / 4 : 1, groups = NG4 * NG4;
  const int g0 = gb * GB;
  const int gcount = min(GB, G - g0);
  const int tl = tid / groups, rem = tid - tl * groups;
  const int ig = rem / NG4, jg = rem - ig * NG4;
  const bool active = (N > 0) && (tl < gcount);

  double *sL = smem;                                             // [GB][EXK][NP]
  double2 *sT = reinterpret_cast<double2 *>(smem + (size_t)GB * EXK * NP);  // [EXK][NP]
  // zero the padding columns once (staging never writes them)
  for (int e = tid; e < GB * EXK * NP; e += blockDim.x) sL[e] = 0.0;
  for (int e = tid; e < EXK * NP; e += blockDim.x) sT[e] = make_double2(0.0, 0.0);
  __syncthreads();

  double2 acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = make_double2(0.0, 0.0);

  const double2 *th = theta + (size_t)w * M * Nt;
  if (N > 0) {
    for (int q0 = 0; q0 < M; q0 += EXK) {
      for (int e = tid; e < gcount * EXK * N; e += blockDim.x) {
        const int gl = e / (EXK * N), rr = e - gl * EXK * N;
        const int qq = rr / N, i = rr - qq * N;
        const int q = q0 + qq;
        sL[((size_t)gl * EXK + qq) * NP + i] =
            (q < M) ? LtT[((size_t)(g0 + gl) * M + q) * Nt + off + i] : 0.0;
      }
      for (int e = tid; e < EXK * N; e += blockDim.x) {
        const int qq = e / N, j = e - qq * N;
        const int q = q0 + qq;
        sT[qq * NP + j] = (q < M) ? th[(size_t)q * Nt + off + j] : make_double2(0.0, 0.0);
      }
      __syncthreads();
      if (active) {
        const double *lrow = sL + (size_t)tl * EXK * NP + ig * 4;
        const double2 *trow = sT + jg * 4;
#pragma unroll 4
        for (int qq = 0; qq < EXK; ++qq) {
          double a[4];
          double2 b[4];
#pragma unroll
          for (int r = 0; r < 4; ++r) a[r] = lrow[qq * NP + r];
#pragma unroll
          for (int c = 0; c < 4; ++c) b[c] = trow[qq * NP + c];
#pragma unroll
          for (int r = 0; r < 4; ++r)
#pragma unroll
            for (int c = 0; c < 4; ++c) {
              acc[r][c].x = fma(a[r], b[c].x, acc[r][c].x);
              acc[r][c].y = fma(a[r], b[c].y, acc[r][c].y);
            }
        }
      }
      __syncthreads();
    }
  }
  // transpose through LDS: sX[tl][i][j] = T_ij
  double2 *sX = reinterpret_cast<double2 *>(smem);
  if (active) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) sX[((size_t)tl * NP + ig * 4 + r) * NP + jg * 4 + c] = acc[r][c];
  }
  __syncthreads();
  double part[2] = {0.0, 0.0};
  if (active) {
#pragma unroll
    for (int r = 0; r < 4; ++r)
#pragma unroll
      for (int c = 0; c < 4; ++c) {
        const int i = ig * 4 + r, j = jg * 4 + c;
        if (i < N && j < N) {
          const double2 t = cmul(acc[r][c], sX[((size_t)tl * NP + j) * NP + i]);
          part[0] += t.x;
          part[1] += t.y;
        }
      }
  }
  block_sum<2>(part, red);
  if (tid == 0) ekpart[((size_t)w * 2 + s) * ngb + gb] = make_double2(-0.5 * part[0], -0.5 * part[1]);
}

// ---- MFMA form ---------------------------------------------------------------
// For one spin block the exchange matrices of all Cholesky vectors and all
// walkers are one real GEMM
//   C[(g, i)][(w, c)] = sum_q Ltilde[g][i][q] * Theta_w[q][c],  c = 2 j + {re, im},
// A = the half-rotated vectors of this spin, stored for this kernel as
// LtS[g][q][NR] (rows i padded with zeros to NR = ceil(N/8)*8), B = the walkers'
// Theta with interleaved complex columns (padded with zeros to CP = 2 NR per walker).
// The four waves of a workgroup form a WY x WX grid: wave (wy, wx) owns GC whole
// Cholesky vectors (RT = GC*NR/16 sixteen-row tiles) of the workgroup's WY*GC
// and one whole walker (CT = CP/16 sixteen-column groups) of its WX, so every
// T^{g}_w is complete inside one wave and the trace needs no other workgroup.
// The K loop stages 16 contraction rows of A and B in LDS with 16-byte loads
// (double-buffered through registers) and issues 4*RT*CT
// v_mfma_f64_4x4x4_4b_f64 per 4 rows: the four blocks of one instruction are
// the four 4-column groups of a 16-column group and share one 4-row slab of A
// (lane 16k+4b+i supplies A_b[i][k], lane 16k+4b+j supplies B_b[k][j], lane
// 16i+4b+j receives D_b[i][j]); on gfx950 this form runs near the FP64 peak.
// Trace: each wave writes T (N x 2N interleaved, row stride 2N+2) to LDS, then
// every lane multiplies the entry it holds, Re T_ij (even column) or Im T_ij
// (odd column), by T_ji read back from LDS:
//   Re sum = sum (Re T_ij Re T_ji - Im T_ij Im T_ji),
//   Im sum = sum (Re T_ij Im T_ji + Im T_ij Re T_ji).
namespace {
constexpr int XKC = 16;     // contraction rows per LDS stage
}  // namespace

template <int NR, int WX>
__global__ __launch_bounds__(kThreads) void k_exchange_mfma(const double *__restrict__ LtS,
                                                           const double *__restrict__ theta, int M, int Nt,
                                                           int off, int N, int G, int W, int stride, int spin,
                                                           double2 *__restrict__ ekpart, double2 *__restrict__ vbpart,
                                                           int ngb, int nwb, int group) {
  constexpr int GC = (NR % 16 == 0) ? 1 : 2;  // Cholesky vectors per wave
  constexpr int WY = 4 / WX;
  constexpr int ROWW = GC * NR;              // rows per wave
  constexpr int RT = ROWW / 16;
  constexpr int CP = 2 * NR;                 // interleaved columns per walker (= ceil(2N/16)*16)
  constexpr int CT = CP / 16;
  constexpr int ROWS = WY * ROWW;            // rows per workgroup
  constexpr int ASZ = XKC * ROWS;            // doubles per A stage
  constexpr int BSZ = WX * XKC * CP;         // doubles per B stage
  constexpr int APT = (ASZ / 2 + kThreads - 1) / kThreads;  // double2 loads per thread
  constexpr int BPT = (BSZ / 2 + kThreads - 1) / kThreads;
  constexpr int TSTRIDE = CP + 2;            // LDS row stride of T (even, breaks bank aliasing)
  extern __shared__ double smem[];
  double *sA = smem;                 // [2][XKC][ROWS]
  double *sB = smem + 2 * ASZ;       // [2][WX][XKC][CP]

  int gb, wb;
  tile_of(blockIdx.x, ngb * nwb, ngb, nwb, group, gb, wb);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wy = wv / WX, wx = wv - (wv / WX) * WX;
  const int g0 = gb * WY * GC, w0 = wb * WX;
  const int twoN = 2 * N;
  const size_t wstride = (size_t)M * Nt * 2;  // doubles per walker

  double2 ra[APT], rb[BPT];
  auto load = [&](int q0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = 2 * (tid + r * kThreads);  // first of two consecutive rows
      const int q = e / ROWS, row = e - q * ROWS;
      const int gl = row / NR, i = row - gl * NR;
      const int g = g0 + gl, gq = q0 + q;
      ra[r] = (e < ASZ && g < G && gq < M)
                  ? *reinterpret_cast<const double2 *>(LtS + ((size_t)g * M + gq) * NR + i)
                  : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = 2 * (tid + r * kThreads);
      const int c = e % CP, t = e / CP;
      const int q = t % XKC, wl = t / XKC;
      const int w = w0 + wl, gq = q0 + q;
      rb[r] = (e < BSZ && c < twoN && w < W && gq < M)
                  ? *reinterpret_cast<const double2 *>(theta + (size_t)w * wstride + (size_t)gq * Nt * 2 + 2 * off + c)
                  : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
    double2 *a = reinterpret_cast<double2 *>(sA + buf * ASZ);
    double2 *b = reinterpret_cast<double2 *>(sB + buf * BSZ);
#pragma unroll
    for (int r = 0; r < APT; ++r)
      if (2 * (tid + r * kThreads) < ASZ) a[tid + r * kThreads] = ra[r];
#pragma unroll
    for (int r = 0; r < BPT; ++r)
      if (2 * (tid + r * kThreads) < BSZ) b[tid + r * kThreads] = rb[r];
  };

  constexpr int TR = 4 * RT;  // 4-row slabs per wave
  double acc[TR][CT];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = 0.0;

  const int nchunk = (M + XKC - 1) / XKC;
  load(0);
  store(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4, l4 = lane & 3;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * XKC);
    const double *a = sA + buf * ASZ + wy * ROWW + l4;
    const double *b = sB + buf * BSZ + wx * XKC * CP + lr;
#pragma unroll
    for (int ks = 0; ks < XKC / 4; ++ks) {
      double av[TR], bv[CT];
#pragma unroll
      for (int i = 0; i < TR; ++i) av[i] = a[(ks * 4 + lk) * ROWS + i * 4];
#pragma unroll
      for (int j = 0; j < CT; ++j) bv[j] = b[(ks * 4 + lk) * CP + j * 16];
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  // Trace, one Cholesky vector of each wave's group at a time.  Padded rows and
  // columns of T are exact zeros (zero rows of LtS, zero columns of B), so the
  // whole NR x CP block is written and read without bounds tests.
  double *sT = smem + (size_t)wv * NR * TSTRIDE;
  const int w = w0 + wx;
  const bool odd = lr & 1;
  double pre = 0.0, pim = 0.0;
  double dg[GC];  // this lane's share of Tr T per Cholesky vector (re or im by column parity)
#pragma unroll
  for (int gl = 0; gl < GC; ++gl) dg[gl] = 0.0;
#pragma unroll
  for (int gl = 0; gl < GC; ++gl) {
    constexpr int SL = NR / 4;  // slabs per Cholesky vector
#pragma unroll
    for (int i = 0; i < SL; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) sT[(i * 4 + lk) * TSTRIDE + j * 16 + lr] = acc[gl * SL + i][j];
    __syncthreads();
#pragma unroll
    for (int i = 0; i < SL; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) {
        const int row = i * 4 + lk, col = j * 16 + lr;
        const double2 tji = *reinterpret_cast<const double2 *>(sT + (col >> 1) * TSTRIDE + 2 * row);
        const double v = acc[gl * SL + i][j];
        pre = fma(v, odd ? -tji.y : tji.x, pre);
        pim = fma(v, odd ? tji.x : tji.y, pim);
        dg[gl] += ((col >> 1) == row) ? v : 0.0;
      }
    __syncthreads();
  }
  pre = wave_sum(pre);
  pim = wave_sum(pim);
  // this spin's part of the force bias, Tr T^{g} = sum_i T_ii: even lanes hold
  // the real parts of the diagonal, odd lanes the imaginary parts
  if (vbpart) {
#pragma unroll
    for (int gl = 0; gl < GC; ++gl) {
      double dre = odd ? 0.0 : dg[gl], dim = odd ? dg[gl] : 0.0;
      dre = wave_sum(dre);
      dim = wave_sum(dim);
      const int g = g0 + wy * GC + gl;
      if (lane == 0 && w < W && g < G) vbpart[((size_t)spin * W + w) * G + g] = make_double2(dre, dim);
    }
  }
  if (lane == 0 && w < W && g0 + wy * GC < G)
    ekpart[((size_t)w * 2 + spin) * stride + gb * WY + wy] = make_double2(-0.5 * pre, -0.5 * pim);
}

namespace {

using ExKernel = void (*)(const double *, const double *, int, int, int, int, int, int, int, int, double2 *,
                          double2 *, int, int, int);

template <int WX>
ExKernel pick_nr(int nr) {
  switch (nr) {
    case 8: return k_exchange_mfma<8, WX>;
    case 16: return k_exchange_mfma<16, WX>;
    case 24: return k_exchange_mfma<24, WX>;
    case 32: return k_exchange_mfma<32, WX>;
    case 40: return k_exchange_mfma<40, WX>;
    case 48: return k_exchange_mfma<48, WX>;
    default: return nullptr;
  }
}

ExKernel pick_exchange(int nr, int wx) {
  switch (wx) {
    case 4: return pick_nr<4>(nr);
    case 2: return pick_nr<2>(nr);
    case 1: return pick_nr<1>(nr);
    default: return nullptr;
  }
}

}  // namespace

ExchangePlan exchange_plan(int N, int G, int wx) {
  ExchangePlan p;
  p.N = N;
  if (N <= 0) return p;
  p.NR = ((N + 7) / 8) * 8;
  p.GC = (p.NR % 16 == 0) ? 1 : 2;
  p.RT = p.GC * p.NR / 16;
  p.CT = p.NR / 8;
  p.WX = wx;
  p.WY = 4 / wx;
  p.ngroups = (G + p.GC - 1) / p.GC;              // one partial per Cholesky-vector group
  p.nwg = (G + p.WY * p.GC - 1) / (p.WY * p.GC);  // workgroups along G
  const size_t stage = 2ull * (XKC * p.WY * p.RT * 16 + p.WX * XKC * p.CT * 16) * sizeof(double);
  const size_t epi = 4ull * p.NR * (2 * p.NR + 2) * sizeof(double);
  p.lds = stage > epi ? stage : epi;
  p.mfma = pick_exchange(p.NR, wx) != nullptr && p.lds <= 160 * 1024;
  if (!p.mfma) p.ngroups = 0;
  return p;
}

hipError_t launch_exchange(const System &s, const double2 *theta, int W, hipStream_t st, double2 *vbpart,
                           int only) {
  if (s.ex_mfma) {
    for (int spin = 0; spin < 2; ++spin) {
      if (only >= 0 && spin != only) continue;
      const ExchangePlan &p = s.ex_plan[spin];
      if (p.N == 0) {
        if (vbpart) {
          hipError_t e = launch_zero2(vbpart + (size_t)spin * W * s.G, (long)W * s.G, st);
          if (e != hipSuccess) return e;
        }
        continue;
      }
      ExKernel k = pick_exchange(p.NR, p.WX);
      const int nwb = (W + p.WX - 1) / p.WX;
      hipLaunchKernelGGL(k, dim3((unsigned)(p.nwg * nwb)), dim3(kThreads), p.lds, st, s.LtS[spin],
                         reinterpret_cast<const double *>(theta), s.M, s.Nt, spin ? s.Na : 0, p.N, s.G, W,
                         s.ex_stride, spin, s.ekpart, vbpart, p.nwg, nwb, s.ex_group);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  if (only == 1) return hipSuccess;  // the VALU kernel covers both spin blocks in one launch
  dim3 grid(s.ex_ngb, 2, W);
  hipLaunchKernelGGL(k_exchange_v1, grid, dim3(kThreads), s.ex_lds, st, s.LtT, theta, s.M, s.Na, s.Nb, s.G,
                     s.ex_gb, s.ex_ngb, s.ekpart);
  return hipGetLastError();
}

__global__ void k_pad_half_rotated(const double *__restrict__ LtT, long rows, int Nt, int off, int N, int NR,
                                   double *__restrict__ LtS) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * NR) return;
  const long r = e / NR;
  const int i = (int)(e - r * NR);
  LtS[e] = (i < N) ? LtT[r * Nt + off + i] : 0.0;
}

hipError_t launch_pad_half_rotated(const double *LtT, int G, int M, int Nt, int off, int N, int NR, double *LtS,
                                   hipStream_t st) {
  const long rows = (long)G * M;
  const long n = rows * NR;
  hipLaunchKernelGGL(k_pad_half_rotated, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, LtT, rows, Nt, off, N,
                     NR, LtS);
  return hipGetLastError();
}

hipError_t exchange_enable_lds(const System &s) {
  if (!s.ex_mfma) return hipSuccess;
  for (int spin = 0; spin < 2; ++spin) {
    const ExchangePlan &p = s.ex_plan[spin];
    if (p.N == 0) continue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pick_exchange(p.NR, p.WX)),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
