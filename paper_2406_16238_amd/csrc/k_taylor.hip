// One term of the Taylor series of the two-body exponential applied to the
// walker slabs (Sec. 2, eq. Bprop, exp(sqrt(dt) V_HS) phi by its series):
//   T_out = alpha * A_w T_in,   tacc += T_out,
// with A_w = sqrt(dt) V_HS of walker w held as real and imaginary M x M planes
// and T complex M x Nt.  As one real product per walker: rows i, columns
// c = (j, re/im) interleaved, contraction over the two planes times q,
//   [Re A | Im A] (M x 2M)  x  [T ; iT] (2M x 2Nt),   iT = (-Im T, Re T).
//
// A workgroup owns BM = 4 WM TR rows and all BN = 16 WN TN >= 2 Nt columns of
// one walker, on a WM x WN grid of waves (4 TR rows x 16 TN columns each), so the
// walker's A rows are read from memory exactly once and its T (M x Nt, 16 M Nt
// bytes) is shared by the M / BM row tiles, which the launch order places on
// one XCD.  Each wave issues TR x TN v_mfma_f64_4x4x4_4b_f64 per 4 contraction
// indices (lane 16k+4b+i supplies A_b[i][k], lane 16k+4b+j supplies B_b[k][j],
// lane 16i+4b+j receives D_b[i][j]; the four blocks are the four 4-column
// groups of one 16-column group).  The contraction is staged 16 indices at a
// time in LDS (k-major, padded rows) with 16-byte global loads, double-buffered
// through registers.  M must be even (16-byte loads of A never straddle the two
// planes) and Nt at most 96; other shapes use the generic GEMM.  The contraction
// starts at kbeg: 0, or M to skip a real plane that is zero (free projection,
// where V_HS is purely imaginary).
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int TKC = 16;  // contraction indices per LDS stage
}

template <int WM, int WN, int TR, int TN>
__global__ __launch_bounds__(64 * WM * WN) void k_taylor_mfma(const double *__restrict__ vhs,
                                                             const double2 *__restrict__ tin,
                                                             double2 *__restrict__ tout, double2 *__restrict__ tacc,
                                                             int M, int Nt, int W, int nrt, double alpha,
                                                             int kbeg) {
  constexpr int NTH = 64 * WM * WN;
  constexpr int BM = WM * 4 * TR, BN = WN * 16 * TN;
  constexpr int LDA = BM + 1, LDB = BN + 1;
  constexpr int AV = BM * TKC / 2;                 // double2 of A per stage
  constexpr int BV = TKC * BN / 2;                 // double2 of B per stage
  constexpr int APT = (AV + NTH - 1) / NTH, BPT = (BV + NTH - 1) / NTH;
  extern __shared__ double tsm[];
  double *sA = tsm;                    // [2][TKC][LDA]
  double *sB = tsm + 2 * TKC * LDA;    // [2][TKC][LDB]

  // contiguous stretch of (walker, row tile) per XCD (workgroups are dealt to
  // the 8 XCDs round-robin), row tile fastest
  const int ntiles = W * nrt;
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int t = x * per + min(x, rem) + jx;
  const int w = t / nrt, i0 = (t - w * nrt) * BM;

  const size_t MM = (size_t)M * M;
  const double *Aw = vhs + (size_t)w * 2 * MM;
  const double2 *Tw = tin + (size_t)w * M * Nt;
  const int K = 2 * M, cols = 2 * Nt;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv - (wv / WN) * WN;
  const int lr = lane & 15, lk = lane >> 4, l4 = lane & 3;

  double2 ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * NTH;                 // (row, k pair)
      const int row = e / (TKC / 2), kp = e - row * (TKC / 2);
      const int gi = i0 + row, gk = k0 + 2 * kp;
      ra[r] = (e < AV && gi < M && gk < K)
                  ? *reinterpret_cast<const double2 *>(Aw + (gk >= M ? MM : 0) + (size_t)gi * M + (gk >= M ? gk - M : gk))
                  : make_double2(0.0, 0.0);
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = tid + r * NTH;                 // (k, complex column j)
      const int kk = e / (BN / 2), j = e - kk * (BN / 2);
      const int gk = k0 + kk;
      double2 v = make_double2(0.0, 0.0);
      if (e < BV && j < Nt && gk < K) {
        const double2 z = Tw[(size_t)(gk >= M ? gk - M : gk) * Nt + j];
        v = gk >= M ? make_double2(-z.y, z.x) : z;
      }
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
    double *a = sA + buf * TKC * LDA;
    double *b = sB + buf * TKC * LDB;
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * NTH;
      if (e < AV) {
        const int row = e / (TKC / 2), kp = e - row * (TKC / 2);
        a[(2 * kp) * LDA + row] = ra[r].x;
        a[(2 * kp + 1) * LDA + row] = ra[r].y;
      }
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = tid + r * NTH;
      if (e < BV) {
        const int kk = e / (BN / 2), j = e - kk * (BN / 2);
        b[kk * LDB + 2 * j] = rb[r].x;
        b[kk * LDB + 2 * j + 1] = rb[r].y;
      }
    }
  };

  constexpr int TRW = TR;  // 4-row slabs per wave
  double acc[TRW][TN];
#pragma unroll
  for (int i = 0; i < TRW; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;

  const int nchunk = (K - kbeg + TKC - 1) / TKC;
  load(kbeg);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load(kbeg + (ch + 1) * TKC);
    const double *a = sA + buf * TKC * LDA + wm * 4 * TR + l4;
    const double *b = sB + buf * TKC * LDB + wn * 16 * TN + lr;
#pragma unroll
    for (int ks = 0; ks < TKC / 4; ++ks) {
      double av[TRW], bv[TN];
#pragma unroll
      for (int i = 0; i < TRW; ++i) av[i] = a[(ks * 4 + lk) * LDA + i * 4];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = b[(ks * 4 + lk) * LDB + j * 16];
#pragma unroll
      for (int i = 0; i < TRW; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  double *to = reinterpret_cast<double *>(tout + (size_t)w * M * Nt);
  double *ta = reinterpret_cast<double *>(tacc + (size_t)w * M * Nt);
#pragma unroll
  for (int i = 0; i < TRW; ++i) {
    const int gi = i0 + wm * 4 * TR + 4 * i + lk;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = wn * 16 * TN + 16 * j + lr;
      if (gi < M && c < cols) {
        const size_t off = (size_t)gi * cols + c;
        const double v = alpha * acc[i][j];
        to[off] = v;
        ta[off] += v;
      }
    }
  }
}

// The same term with three real products instead of four (the 3M form of a
// complex product): with A = Ar + i Ai and T = Tr + i Ti,
//   P1 = Ar Tr,  P2 = Ai Ti,  P3 = (Ar + Ai)(Tr + Ti),
//   A T = (P1 - P2) + i (P3 - P1 - P2),
// each an M x M by M x Nt real product, so a term costs 6 M^2 Nt flops instead
// of 8.  A workgroup owns BM = 4 WM TR rows and BNC = 16 WN TN >= Nt complex
// columns of one walker; wave (wm, wn) holds the three products of its
// 4 TR x 16 TN block, so the combination happens in registers and each lane
// writes whole complex entries.  Ar + Ai and Tr + Ti are formed from the
// staged operands in registers.  LDS per stage: the Ar and Ai rows (k-major)
// and the Tr and Ti planes of 16 contraction indices.
// IMAG: A = i Ai (free projection, a real-field V_HS): A T = -Ai Ti + i Ai Tr,
// two products P1 = Ai Tr, P2 = Ai Ti and only the Ai rows staged.
template <int WM, int WN, int TR, int TN, bool IMAG = false>
__global__ __launch_bounds__(64 * WM * WN, 2) void k_taylor3m(const double *__restrict__ vhs,
                                                             const double2 *__restrict__ tin,
                                                             double2 *__restrict__ tout,
                                                             double2 *__restrict__ tacc, int M, int Nt, int W,
                                                             int nrt, double alpha) {
  constexpr int NTH = 64 * WM * WN;
  constexpr int BM = WM * 4 * TR, BNC = WN * 16 * TN;
  constexpr int LDA = BM + 1, LDB = BNC + 1;
  constexpr int NPL = IMAG ? 1 : 2;                 // staged planes of A
  constexpr int AV = NPL * BM * TKC / 2;            // double2 (k pairs) of A per stage
  constexpr int BV = TKC * BNC;                     // complex entries of T per stage
  constexpr int APT = (AV + NTH - 1) / NTH, BPT = (BV + NTH - 1) / NTH;
  extern __shared__ double tsm[];
  double *sA = tsm;                          // [2 buf][NPL plane][TKC][LDA]
  double *sB = tsm + 2 * NPL * TKC * LDA;    // [2 buf][2 plane][TKC][LDB]

  const int ntiles = W * nrt;
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int t = x * per + min(x, rem) + jx;
  const int w = t / nrt, i0 = (t - w * nrt) * BM;

  const size_t MM = (size_t)M * M;
  const double *Aw = vhs + (size_t)w * 2 * MM;
  const double2 *Tw = tin + (size_t)w * M * Nt;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv - (wv / WN) * WN;
  const int lr = lane & 15, lk = lane >> 4, l4 = lane & 3;

  // Loop-invariant addressing: A element (plane, row, k pair) e = tid + NTH r
  // keeps its source offset at k = 0 and its LDS slot; T is loaded as columns
  // t%16 + 16c of contraction row t/16.  Interior chunks skip the bounds tests.
  static_assert(BPT * NTH == BV && NTH == 16 * TKC, "T staged as t%16 + 16c, row t/16");
  const int tq = tid >> 4, tl = tid & 15;
  size_t offa[APT];
  int sla[APT];
  bool rowa[APT];
#pragma unroll
  for (int r = 0; r < APT; ++r) {
    const int e = tid + r * NTH;                   // (plane, row, k pair)
    const int pr = e / (TKC / 2), kp = e - pr * (TKC / 2);
    const int pl = pr / BM, row = pr - pl * BM;
    offa[r] = (IMAG ? 1 : pl) * MM + (size_t)(i0 + row) * M + 2 * kp;
    sla[r] = (pl * TKC + 2 * kp) * LDA + row;
    rowa[r] = e < AV && i0 + row < M;
  }
  const bool rows_in = i0 + BM <= M && AV % NTH == 0, cols_in = BNC <= Nt;
  const int kpl = 2 * ((tid % (TKC / 2)));         // the k pair of every A element of this thread

  double2 ra[APT], rb[BPT];
  auto load = [&](int k0) {
    const double2 *pb = Tw + (size_t)(k0 + tq) * Nt + tl;
    if (rows_in && cols_in && k0 + TKC <= M) {
#pragma unroll
      for (int r = 0; r < APT; ++r) ra[r] = *reinterpret_cast<const double2 *>(Aw + offa[r] + k0);
#pragma unroll
      for (int c = 0; c < BPT; ++c) rb[c] = pb[16 * c];
    } else {
      const bool ka = k0 + kpl < M, kb = k0 + tq < M;
#pragma unroll
      for (int r = 0; r < APT; ++r)
        ra[r] = (rowa[r] && ka) ? *reinterpret_cast<const double2 *>(Aw + offa[r] + k0) : make_double2(0.0, 0.0);
#pragma unroll
      for (int c = 0; c < BPT; ++c) rb[c] = (kb && tl + 16 * c < Nt) ? pb[16 * c] : make_double2(0.0, 0.0);
    }
  };
  auto store = [&](int buf) {
    double *a = sA + buf * NPL * TKC * LDA;
    double *b = sB + buf * 2 * TKC * LDB;
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      if (AV % NTH == 0 || tid + r * NTH < AV) {
        a[sla[r]] = ra[r].x;
        a[sla[r] + LDA] = ra[r].y;
      }
    }
#pragma unroll
    for (int c = 0; c < BPT; ++c) {
      b[tq * LDB + tl + 16 * c] = rb[c].x;
      b[(TKC + tq) * LDB + tl + 16 * c] = rb[c].y;
    }
  };

  double p1[TR][TN], p2[TR][TN], p3[TR][TN];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) p1[i][j] = p2[i][j] = p3[i][j] = 0.0;

  const int nchunk = (M + TKC - 1) / TKC;
  // a wave of the last row tile whose rows all lie past M stages operands with
  // the others but issues no MFMA
  const bool live = i0 + wm * 4 * TR < M;
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * TKC);
    const double *ar = sA + buf * NPL * TKC * LDA + wm * 4 * TR + l4;
    const double *ai = IMAG ? ar : ar + TKC * LDA;
    const double *br = sB + buf * 2 * TKC * LDB + wn * 16 * TN + lr;
    const double *bi = br + TKC * LDB;
#pragma unroll
    for (int ks = 0; ks < (live ? TKC / 4 : 0); ++ks) {
      const int kr = ks * 4 + lk;
      double xr[TR], xi[TR], yr[TN], yi[TN];
#pragma unroll
      for (int i = 0; i < TR; ++i) {
        xi[i] = ai[kr * LDA + i * 4];
        xr[i] = IMAG ? 0.0 : ar[kr * LDA + i * 4];
      }
#pragma unroll
      for (int j = 0; j < TN; ++j) {
        yr[j] = br[kr * LDB + j * 16];
        yi[j] = bi[kr * LDB + j * 16];
      }
      if constexpr (IMAG) {
#pragma unroll
        for (int i = 0; i < TR; ++i)
#pragma unroll
          for (int j = 0; j < TN; ++j) {
            p1[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi[i], yr[j], p1[i][j], 0, 0, 0);
            p2[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xi[i], yi[j], p2[i][j], 0, 0, 0);
          }
        continue;
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
        for (int j = 0; j < TN; ++j) p3[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(xr[i], yr[j], p3[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  double2 *to = tout + (size_t)w * M * Nt;
  double2 *ta = tacc + (size_t)w * M * Nt;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int gi = i0 + wm * 4 * TR + 4 * i + lk;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int c = wn * 16 * TN + 16 * j + lr;
      if (gi < M && c < Nt) {
        const size_t off = (size_t)gi * Nt + c;
        const double re = IMAG ? -p2[i][j] : p1[i][j] - p2[i][j];
        const double im = IMAG ? p1[i][j] : (p3[i][j] - p1[i][j]) - p2[i][j];
        const double2 v = make_double2(alpha * re, alpha * im);
        to[off] = v;
        const double2 o = ta[off];
        ta[off] = make_double2(o.x + v.x, o.y + v.y);
      }
    }
  }
}

namespace {
template <int WM, int WN, int TR, int TN>
hipError_t run_taylor(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st,
                      int kbeg) {
  constexpr int BM = WM * 4 * TR, BN = WN * 16 * TN;
  static_assert(BN >= 2, "columns");
  const size_t lds = 2ull * TKC * ((BM + 1) + (BN + 1)) * sizeof(double);
  auto k = k_taylor_mfma<WM, WN, TR, TN>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int nrt = (s.M + BM - 1) / BM;
  hipLaunchKernelGGL(k, dim3((unsigned)(W * nrt)), dim3(64 * WM * WN), lds, st, s.vhs, tin, tout, s.tacc, s.M, s.Nt,
                     W, nrt, alpha, kbeg);
  return hipGetLastError();
}
}  // namespace

namespace {
template <int WM, int WN, int TR, int TN, bool IMAG = false>
hipError_t run_taylor3m(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st) {
  constexpr int BM = WM * 4 * TR, BNC = WN * 16 * TN;
  const size_t lds = 2ull * TKC * ((IMAG ? 1 : 2) * (BM + 1) + 2 * (BNC + 1)) * sizeof(double);
  auto k = k_taylor3m<WM, WN, TR, TN, IMAG>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  const int nrt = (s.M + BM - 1) / BM;
  hipLaunchKernelGGL(k, dim3((unsigned)(W * nrt)), dim3(64 * WM * WN), lds, st, s.vhs, tin, tout, s.tacc, s.M, s.Nt,
                     W, nrt, alpha);
  return hipGetLastError();
}

template <int TR, bool IMAG = false>
hipError_t run_taylor3m_tn(const System &s, const double2 *tin, double2 *tout, double alpha, int W, hipStream_t st) {
  switch ((s.Nt + 15) / 16) {
    case 1: return run_taylor3m<4, 1, TR, 1, IMAG>(s, tin, tout, alpha, W, st);
    case 2: return run_taylor3m<4, 1, TR, 2, IMAG>(s, tin, tout, alpha, W, st);
    case 3: return run_taylor3m<4, 1, TR, 3, IMAG>(s, tin, tout, alpha, W, st);
    case 4: return run_taylor3m<4, 1, TR, 4, IMAG>(s, tin, tout, alpha, W, st);
    case 5: return run_taylor3m<4, 1, TR, 5, IMAG>(s, tin, tout, alpha, W, st);
    // 96 columns: 32-row tiles keep the three accumulator sets in registers
    default: return run_taylor3m<4, 1, 2, 6, IMAG>(s, tin, tout, alpha, W, st);
  }
}
}  // namespace

bool taylor_mfma_supported(int M, int Nt) { return M % 2 == 0 && Nt >= 1 && Nt <= 96; }

hipError_t launch_taylor_mfma(const System &s, const double2 *tin, double2 *tout, double alpha, int W,
                              hipStream_t st, int kbeg) {
  // a complex V_HS: three real products per term (taylor4, or variants 1..8,
  // keep the four-product kernel for comparison runs; 9..10 other 3M row tiles)
  if (!s.taylor4 && (s.taylor_variant == 0 || s.taylor_variant >= 9)) {
    if (kbeg != 0) {
      // purely imaginary V_HS (its real plane is not formed): two products
      if (kbeg != s.M) return hipErrorInvalidValue;
      return s.taylor_variant == 10 ? run_taylor3m_tn<4, true>(s, tin, tout, alpha, W, st)
                                    : run_taylor3m_tn<3, true>(s, tin, tout, alpha, W, st);
    }
    switch (s.taylor_variant) {
      case 9: return run_taylor3m_tn<2>(s, tin, tout, alpha, W, st);
      case 10: return run_taylor3m_tn<4>(s, tin, tout, alpha, W, st);
      default: return run_taylor3m_tn<3>(s, tin, tout, alpha, W, st);
    }
  }
  if (s.Nt <= 16) return run_taylor<2, 2, 16, 1>(s, tin, tout, alpha, W, st, kbeg);
  if (s.Nt <= 32) return run_taylor<2, 2, 16, 2>(s, tin, tout, alpha, W, st, kbeg);
  if (s.Nt <= 48) return run_taylor<2, 2, 12, 3>(s, tin, tout, alpha, W, st, kbeg);
  if (s.Nt <= 64) return run_taylor<2, 2, 12, 4>(s, tin, tout, alpha, W, st, kbeg);
  if (s.Nt <= 80) {
    switch (s.taylor_variant) {
      case 1: return run_taylor<2, 1, 10, 10>(s, tin, tout, alpha, W, st, kbeg);
      case 2: return run_taylor<1, 2, 20, 5>(s, tin, tout, alpha, W, st, kbeg);
      case 3: return run_taylor<2, 2, 20, 5>(s, tin, tout, alpha, W, st, kbeg);
      case 4: return run_taylor<4, 1, 5, 10>(s, tin, tout, alpha, W, st, kbeg);
      case 5: return run_taylor<2, 2, 10, 5>(s, tin, tout, alpha, W, st, kbeg);
      case 6: return run_taylor<2, 2, 4, 5>(s, tin, tout, alpha, W, st, kbeg);
      case 7: return run_taylor<2, 2, 7, 5>(s, tin, tout, alpha, W, st, kbeg);
      case 8: return run_taylor<2, 2, 8, 5>(s, tin, tout, alpha, W, st, kbeg);
      // default 48-row tiles: at the headline shape 0.82 ms per term against
      // 0.93 for 80 rows (a shorter grid tail at three waves per SIMD)
      default: return run_taylor<2, 2, 6, 5>(s, tin, tout, alpha, W, st, kbeg);
    }
  }
  return run_taylor<2, 2, 8, 6>(s, tin, tout, alpha, W, st, kbeg);
}

}  // namespace afqmc
