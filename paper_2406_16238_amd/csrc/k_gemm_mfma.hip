// FP64 MFMA GEMM for the dense contractions of the propagation step.
//
//   C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j)   [and C2(i,j) += that value]
//
// Workgroup tile BM x BN = (WM*TM*16) x (WN*TN*16) on a WM x WN grid of waves.
// Each wave issues v_mfma_f64_4x4x4_4b_f64 (four independent 4x4x4 products per
// instruction; on gfx950 it sustains close to the FP64 peak, about 1.6x the
// 16x16x4 form): the four blocks are four 4-column groups of one 16-column
// group, all sharing one 4-row slab of A.  Lane layout: lane 16k+4b+i supplies
// A_b[i][k], lane 16k+4b+j supplies B_b[k][j], lane 16i+4b+j receives D_b[i][j],
// so a B operand is 16 consecutive columns of one k row per lane group and the
// result of slab r, group c sits at row 4r + lane/16, column 16c + lane%16.
// A wave owns 4*TM x TN such accumulators.  The K loop stages 16 contraction
// indices of A and B in LDS (k-major), double-buffered through registers.
// Operand access modes:
//   A mode 0: A(i,k) = A[i*sai + k]                (k contiguous)
//   A mode 1: A(i,k) = A[i + k*sak]                (i contiguous)
//   A mode 2: k < kh: A[i*sai + k]; k >= kh: A[aplane + i*sai + k - kh]
//             (a complex matrix held as real and imaginary planes, with the
//              contraction running over both: [Re A | Im A])
//   A mode 3: A(i,k) = A[(i/2)*sai + 2k + i%2]      (rows = interleaved complex
//             vectors stored one after another: walker slabs read as (re, im))
//   B mode 0: B(k,j) = B[k*sbk + j]                (j contiguous)
//   B mode 1: B(k,j) = B[k + j*sbj]                (k contiguous)
//   B mode 3: k < kh: B[k*sbk + j]; k >= kh: the same row of the complex matrix
//             multiplied by i, (re, im) -> (-im, re)  ([T ; iT] for [Re A | Im A])
// With cplx_rows set, output row i goes to C[(i/2)*sci + i%2 + j*scj] (the two
// rows of one complex vector interleave).
// The launch is 1-D over (tile, batch, K slice) and remapped so that each XCD
// (every 8th workgroup id) walks one contiguous stretch of that order, row tiles
// fastest: a B column panel stays in one XCD's L2 while all row tiles consume
// it, and the tiles of one batch entry (one walker's slab) share an XCD.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int MKC = 16;
}

template <int WM, int WN, int TM, int TN, int AMODE, int BMODE, int MINB>
__global__ __launch_bounds__(kThreads, MINB) void k_gemm_mfma(GemmArgs a, int kchunk, int gx, int gy) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  constexpr int LDA = BM + 1, LDB = BN + 1;     // padded LDS rows
  constexpr int APT = (AMODE == 3) ? BM * MKC / (2 * kThreads) : BM * MKC / kThreads;
  constexpr int BPT = BN * MKC / kThreads;
  static_assert(WM * WN == 4, "four waves");
  static_assert(!(AMODE == 0 && BMODE == 0) || (MKC == 16 && kThreads == 256 && APT * 16 == BM && BPT * 16 == BN),
                "load00 covers the tiles");
  extern __shared__ double smem[];
  double *sA = smem;                        // [2][MKC][LDA]
  double *sB = smem + 2 * MKC * LDA;        // [2][MKC][LDB]

  // XCD-aware order over (tile, batch entry and K slice)
  const int nb = gx * gy;
  const int ntot = gridDim.x;
  const int per = ntot >> 3, rem = ntot & 7;
  const int xcd = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int lin = xcd * per + min(xcd, rem) + jx;
  const int tile = lin % nb, bz = lin / nb;
  const int bx = tile % gx, by = tile / gx;
  const int i0 = bx * BM, j0 = by * BN;
  const int b = bz / a.ksplit, s = bz - b * a.ksplit;
  const int kbeg = s * kchunk;
  const int kend = min(a.k, kbeg + kchunk);
  const double *A = a.A + (size_t)b * a.sab;
  const double *B = a.B + (size_t)b * a.sbb;

  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv / WN, wn = wv - (wv / WN) * WN;
  const int lr = lane & 15, lk = lane >> 4;

  double ra[(AMODE == 3) ? 2 * APT : APT];
  double rb[BPT];
  // Modes 0/0 (row-major A and B): thread t loads A rows t/16 + 16r at k = t%16
  // and B columns t%16 + 16c at k row t/16, so every address is a per-thread
  // base plus a uniform step; interior chunks skip the bounds tests.
  const int tq = tid >> 4, tl = tid & 15;
  auto load00 = [&](int k0) {
    const double *pa = A + (size_t)(i0 + tq) * a.sai + k0 + tl;
    const double *pb = B + (size_t)(k0 + tq) * a.sbk + j0 + tl;
    const size_t astep = (size_t)16 * a.sai;
    if (i0 + BM <= a.m && j0 + BN <= a.n && k0 + MKC <= kend) {
#pragma unroll
      for (int r = 0; r < APT; ++r) ra[r] = pa[r * astep];
#pragma unroll
      for (int c = 0; c < BPT; ++c) rb[c] = pb[16 * c];
    } else {
      const bool ka = k0 + tl < kend, kb = k0 + tq < kend;
#pragma unroll
      for (int r = 0; r < APT; ++r) ra[r] = (ka && i0 + tq + 16 * r < a.m) ? pa[r * astep] : 0.0;
#pragma unroll
      for (int c = 0; c < BPT; ++c) rb[c] = (kb && j0 + tl + 16 * c < a.n) ? pb[16 * c] : 0.0;
    }
  };
  auto load = [&](int k0) {
    if constexpr (AMODE == 0 && BMODE == 0) {
      load00(k0);
      return;
    }
    if (AMODE == 3) {
#pragma unroll
      for (int r = 0; r < APT; ++r) {
        const int e = tid + r * kThreads;
        const int kk = e % MKC, wl = e / MKC;
        const int gi = i0 + 2 * wl, gk = k0 + kk;
        double2 v = make_double2(0.0, 0.0);
        if (gi < a.m && gk < kend) v = *reinterpret_cast<const double2 *>(A + (size_t)(gi / 2) * a.sai + 2 * (size_t)gk);
        ra[2 * r] = v.x;
        ra[2 * r + 1] = v.y;
      }
    } else
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * kThreads;
      int ii, kk;
      if (AMODE == 1) { ii = e % BM; kk = e / BM; }
      else { kk = e % MKC; ii = e / MKC; }
      const int gi = i0 + ii, gk = k0 + kk;
      double v = 0.0;
      if (gi < a.m && gk < kend) {
        if (AMODE == 0) v = A[(size_t)gi * a.sai + gk];
        else if (AMODE == 1) v = A[(size_t)gi + (size_t)gk * a.sak];
        else v = (gk < a.khalf) ? A[(size_t)gi * a.sai + gk] : A[a.aplane + (size_t)gi * a.sai + (gk - a.khalf)];
      }
      ra[r] = v;
    }
    {
#pragma unroll
      for (int r = 0; r < BPT; ++r) {
        const int e = tid + r * kThreads;
        int jj, kk;
        if (BMODE == 1) { kk = e % MKC; jj = e / MKC; }
        else { jj = e % BN; kk = e / BN; }
        const int gj = j0 + jj, gk = k0 + kk;
        double v = 0.0;
        if (gj < a.n && gk < kend) {
          if (BMODE == 0) v = B[(size_t)gk * a.sbk + gj];
          else if (BMODE == 1) v = B[(size_t)gk + (size_t)gj * a.sbj];
          else {
            if (gk < a.khalf) v = B[(size_t)gk * a.sbk + gj];
            else {
              const size_t row = (size_t)(gk - a.khalf) * a.sbk;
              v = (gj & 1) ? B[row + gj - 1] : -B[row + gj + 1];
            }
          }
        }
        rb[r] = v;
      }
    }
  };
  auto store = [&](int buf) {
    double *sa = sA + buf * MKC * LDA;
    double *sb = sB + buf * MKC * LDB;
    if constexpr (AMODE == 0 && BMODE == 0) {
#pragma unroll
      for (int r = 0; r < APT; ++r) sa[tl * LDA + tq + 16 * r] = ra[r];
#pragma unroll
      for (int c = 0; c < BPT; ++c) sb[tq * LDB + tl + 16 * c] = rb[c];
      return;
    }
    if (AMODE == 3) {
#pragma unroll
      for (int r = 0; r < APT; ++r) {
        const int e = tid + r * kThreads;
        const int kk = e % MKC, wl = e / MKC;
        sa[kk * LDA + 2 * wl] = ra[2 * r];
        sa[kk * LDA + 2 * wl + 1] = ra[2 * r + 1];
      }
    } else {
#pragma unroll
      for (int r = 0; r < APT; ++r) {
        const int e = tid + r * kThreads;
        int ii, kk;
        if (AMODE == 1) { ii = e % BM; kk = e / BM; }
        else { kk = e % MKC; ii = e / MKC; }
        sa[kk * LDA + ii] = ra[r];
      }
    }
    {
#pragma unroll
      for (int r = 0; r < BPT; ++r) {
        const int e = tid + r * kThreads;
        int jj, kk;
        if (BMODE == 1) { kk = e % MKC; jj = e / MKC; }
        else { jj = e % BN; kk = e / BN; }
        sb[kk * LDB + jj] = rb[r];
      }
    }
  };

  constexpr int TR = 4 * TM;  // 4-row slabs per wave
  double acc[TR][TN];
#pragma unroll
  for (int i = 0; i < TR; ++i)
#pragma unroll
    for (int j = 0; j < TN; ++j) acc[i][j] = 0.0;
  const int l4 = lane & 3;

  const int nchunk = (kend - kbeg + MKC - 1) / MKC;
  if (nchunk > 0) {
    load(kbeg);
    store(0);
  }
  __syncthreads();
  // a wave whose rows (or columns) all lie past the edge of C stages operands
  // with the others but issues no MFMA
  const bool live = i0 + wm * TM * 16 < a.m && j0 + wn * TN * 16 < a.n;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load(kbeg + (ch + 1) * MKC);
    const double *sa = sA + buf * MKC * LDA + wm * TM * 16 + l4;
    const double *sb = sB + buf * MKC * LDB + wn * TN * 16 + lr;
#pragma unroll
    for (int ks = 0; ks < (live ? MKC / 4 : 0); ++ks) {
      double av[TR], bv[TN];
#pragma unroll
      for (int i = 0; i < TR; ++i) av[i] = sa[(ks * 4 + lk) * LDA + i * 4];
#pragma unroll
      for (int j = 0; j < TN; ++j) bv[j] = sb[(ks * 4 + lk) * LDB + j * 16];
#pragma unroll
      for (int i = 0; i < TR; ++i)
#pragma unroll
        for (int j = 0; j < TN; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_4x4x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  double *C = a.C + (size_t)b * a.scb + (size_t)s * a.scs;
  double *C2 = a.C2 ? a.C2 + (size_t)b * a.scb : nullptr;
#pragma unroll
  for (int i = 0; i < TR; ++i) {
    const int gi = i0 + wm * TM * 16 + i * 4 + lk;
#pragma unroll
    for (int j = 0; j < TN; ++j) {
      const int gj = j0 + wn * TN * 16 + j * 16 + lr;
      if (gj >= a.n || gi >= a.m) continue;
      const size_t off = (a.cplx_rows ? (size_t)(gi >> 1) * a.sci + (gi & 1) : (size_t)gi * a.sci) +
                         (size_t)gj * a.scj;
      double v = a.alpha * acc[i][j];
      if (a.beta != 0.0) v = fma(a.beta, C[off], v);
      C[off] = v;
      if (C2) C2[off] += v;
    }
  }
}

namespace {

template <int WM, int WN, int TM, int TN, int AMODE, int BMODE, int MINB = 1>
hipError_t run(const GemmArgs &a, hipStream_t st) {
  constexpr int BM = WM * TM * 16, BN = WN * TN * 16;
  const int ks = a.ksplit < 1 ? 1 : a.ksplit;
  int kchunk = (a.k + ks - 1) / ks;
  kchunk = ((kchunk + MKC - 1) / MKC) * MKC;
  GemmArgs g = a;
  g.ksplit = ks;
  const int gx = (a.m + BM - 1) / BM, gy = (a.n + BN - 1) / BN;
  const size_t lds = (size_t)2 * MKC * ((BM + 1) + (BN + 1)) * sizeof(double);
  auto k = k_gemm_mfma<WM, WN, TM, TN, AMODE, BMODE, MINB>;
  static bool attr = false;
  if (!attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k), hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  hipLaunchKernelGGL(k, dim3((unsigned)((long)gx * gy * a.batch * ks)), dim3(kThreads), lds, st, g, kchunk, gx, gy);
  return hipGetLastError();
}

}  // namespace

// V_HS planes: rows (w, c) = 2W, columns M^2 (or the packed M(M+1)/2),
// contraction over G.  Default: 128 x 128 tiles, 64 x 64 per wave, two waves
// per SIMD (245 registers since the operand loads became affine; measured 7 %
// faster at the headline shape than 128 x 96 tiles).
hipError_t gemm_vhs_mfma(const GemmArgs &a, hipStream_t st, int shape) {
  // rows x columns of a workgroup tile: 128 x 128 (default), 128 x 96,
  // 64 x 128 and 128 x 64, all at two waves per SIMD; the set-up tuner times
  // them per problem shape
  switch (shape) {
    case 1: return run<2, 2, 4, 3, 0, 0, 2>(a, st);
    case 2: return run<2, 2, 2, 4, 0, 0, 2>(a, st);
    case 3: return run<4, 1, 2, 4, 0, 0, 2>(a, st);
    default: return run<2, 2, 4, 4, 0, 0, 2>(a, st);
  }
}
// B1 times walker slabs: M rows, 2 Nt real columns, batched over walkers.
hipError_t gemm_b1_mfma(const GemmArgs &a, hipStream_t st) { return run<4, 1, 1, 5, 0, 0>(a, st); }
// Taylor term: [Re A | Im A] times [T ; iT], batched over walkers.
hipError_t gemm_taylor_mfma(const GemmArgs &a, hipStream_t st) { return run<4, 1, 1, 5, 2, 3>(a, st); }
// Force bias: walker rows (interleaved complex) times Ltilde columns, split-K.
hipError_t gemm_fb_mfma(const GemmArgs &a, hipStream_t st) { return run<2, 2, 2, 2, 3, 1>(a, st); }
// Generic square-ish products of set-up (row-major, no transposes).
hipError_t gemm_nn_mfma(const GemmArgs &a, hipStream_t st) { return run<2, 2, 2, 2, 0, 0>(a, st); }

}  // namespace afqmc
