// FP64 contraction kernels of the propagation step and of set-up:
//  * a strided, batched, split-K real GEMM (LDS-tiled, 64x64 tiles, 4x4 register
//    micro-tiles per thread) used for the force bias, the two-body generator
//    V_HS, the one-body factor B1 and the set-up products;
//  * the complex Taylor-term product t' = alpha A_w t with A_w = sqrt(dt) V_HS
//    held as real/imaginary planes (Sec. 2, eq. Bprop: exp(-sqrt(dt) y.v) acts
//    on the orbitals as the matrix exponential of sqrt(dt) V_HS).
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int TBM = 64, TBN = 64, TBK = 16;
}

__global__ __launch_bounds__(kThreads) void k_gemm_f64(GemmArgs a, int kchunk) {
  __shared__ double As[TBK][TBM + 4];
  __shared__ double Bs[TBK][TBN + 4];
  const int tid = threadIdx.x;
  const int tx = tid & 15, ty = tid >> 4;
  const int j0 = blockIdx.x * TBN, i0 = blockIdx.y * TBM;
  const int bz = blockIdx.z;
  const int b = bz / a.ksplit, s = bz - b * a.ksplit;
  const int kbeg = s * kchunk;
  const int kend = min(a.k, kbeg + kchunk);
  const double *A = a.A + (size_t)b * a.sab;
  const double *B = a.B + (size_t)b * a.sbb;
  const bool a_kfast = (a.sak == 1);
  const bool b_jfast = (a.sbj == 1);

  double acc[4][4];
#pragma unroll
  for (int r = 0; r < 4; ++r)
#pragma unroll
    for (int c = 0; c < 4; ++c) acc[r][c] = 0.0;

  for (int k0 = kbeg; k0 < kend; k0 += TBK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int ii, kk;
      if (a_kfast) { kk = tid & 15; ii = (tid >> 4) + 16 * r; }
      else { ii = tid & 63; kk = (tid >> 6) + 4 * r; }
      const int gi = i0 + ii, gk = k0 + kk;
      As[kk][ii] = (gi < a.m && gk < kend) ? A[(size_t)gi * a.sai + (size_t)gk * a.sak] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      int jj, kk;
      if (b_jfast) { jj = tid & 63; kk = (tid >> 6) + 4 * r; }
      else { kk = tid & 15; jj = (tid >> 4) + 16 * r; }
      const int gj = j0 + jj, gk = k0 + kk;
      Bs[kk][jj] = (gj < a.n && gk < kend) ? B[(size_t)gk * a.sbk + (size_t)gj * a.sbj] : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TBK; ++kk) {
      double av[4], bv[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) av[r] = As[kk][ty * 4 + r];
#pragma unroll
      for (int c = 0; c < 4; ++c) bv[c] = Bs[kk][tx * 4 + c];
#pragma unroll
      for (int r = 0; r < 4; ++r)
#pragma unroll
        for (int c = 0; c < 4; ++c) acc[r][c] = fma(av[r], bv[c], acc[r][c]);
    }
    __syncthreads();
  }

  double *C = a.C + (size_t)b * a.scb + (size_t)s * a.scs;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gi = i0 + ty * 4 + r;
    if (gi >= a.m) continue;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
      const int gj = j0 + tx * 4 + c;
      if (gj >= a.n) continue;
      double *p = C + (size_t)gi * a.sci + (size_t)gj * a.scj;
      const double v = a.alpha * acc[r][c];
      *p = (a.beta != 0.0) ? fma(a.beta, *p, v) : v;
    }
  }
}

hipError_t gemm_f64(const GemmArgs &a, hipStream_t st) {
  if (a.m <= 0 || a.n <= 0 || a.batch <= 0) return hipSuccess;
  const int ks = a.ksplit < 1 ? 1 : a.ksplit;
  int kchunk = (a.k + ks - 1) / ks;
  kchunk = ((kchunk + TBK - 1) / TBK) * TBK;
  GemmArgs b = a;
  b.ksplit = ks;
  dim3 grid((a.n + TBN - 1) / TBN, (a.m + TBM - 1) / TBM, a.batch * ks);
  hipLaunchKernelGGL(k_gemm_f64, grid, dim3(kThreads), 0, st, b, kchunk);
  return hipGetLastError();
}

// ---- force bias: vbias[w][g] = sum_k LtT[g][k] Theta[w][k], k = (q, i') -----
// MFMA form: rows (w, re/im) of the walker slabs times the half-rotated vectors,
// split over K; VALU form: the strided GEMM above with the roles swapped.
hipError_t launch_force_bias_gemm(const System &s, const double2 *theta, int W, hipStream_t st) {
  const long K = (long)s.M * s.Nt;
  GemmArgs a;
  if (s.use_mfma_gemm) {
    a.m = 2 * W; a.n = s.G; a.k = (int)K; a.ksplit = s.fb_ksplit;
    a.A = reinterpret_cast<const double *>(theta); a.sai = 2 * K;
    a.B = s.LtT; a.sbj = K;
    a.C = reinterpret_cast<double *>(s.fbpart); a.sci = 2L * s.G; a.scj = 2; a.scs = 2L * W * s.G;
    a.cplx_rows = 1;
    return gemm_fb_mfma(a, st);
  }
  a.m = s.G; a.n = W; a.k = (int)K; a.batch = 2; a.ksplit = s.fb_ksplit;
  a.A = s.LtT; a.sai = K; a.sak = 1; a.sab = 0;
  a.B = reinterpret_cast<const double *>(theta); a.sbk = 2; a.sbj = 2 * K; a.sbb = 1;
  a.C = reinterpret_cast<double *>(s.fbpart); a.sci = 2; a.scj = 2L * s.G; a.scb = 1;
  a.scs = 2L * W * s.G;
  return gemm_f64(a, st);
}

// ---- two-body generator: vhs[w][c][pq] = sum_g yp[w][c][g] L[g][pq] ----------
// The L^g are symmetric, so is every V_HS: with the packed upper triangles
// (Lp[g][t], t over p <= q row by row: the packed Cholesky vectors of Sec. 3.2)
// the product runs over M(M+1)/2 columns instead of M^2, and a second kernel
// writes each packed element to (p, q) and (q, p).  Each element is the same
// sum over g in the same order as in the unpacked product.

// t0(p) = index of element (p, p) in the packed rows: p M - p (p - 1) / 2.
__device__ __forceinline__ long packed_row(long p, long M) { return p * M - p * (p - 1) / 2; }

// Lp[g][t] = L[g][p][q] for p <= q.  Grid (rows p, G); block over q.
__global__ void k_pack_upper(const double *__restrict__ L, int M, double *__restrict__ Lp) {
  const int p = blockIdx.x, g = blockIdx.y;
  const long Mp = (long)M * (M + 1) / 2;
  const double *src = L + ((size_t)g * M + p) * M;
  double *dst = Lp + (size_t)g * Mp + packed_row(p, M) - p;
  for (int q = p + threadIdx.x; q < M; q += blockDim.x) dst[q] = src[q];
}

// full[m][p][q] = full[m][q][p] = packed[m][t(p, q)] for p <= q; one workgroup
// per 32 x 32 tile (bi <= bj) of one matrix m, the transposed copy through LDS.
__global__ __launch_bounds__(kThreads) void k_unpack_symmetric(const double *__restrict__ packed, int M, int ntile,
                                                               int pstride, int poff, double *__restrict__ full) {
  __shared__ double tile[32][33];
  const int m = blockIdx.y * pstride + poff;
  // tile index -> (bi, bj), bi <= bj, row-major over the upper triangle of tiles
  int t = blockIdx.x, bi = 0;
  while (t >= ntile - bi) {
    t -= ntile - bi;
    ++bi;
  }
  const int bj = bi + t;
  const long Mp = (long)M * (M + 1) / 2;
  const double *P = packed + (size_t)m * Mp;
  double *F = full + (size_t)m * M * M;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;  // 32 x 8
  for (int r = ty; r < 32; r += 8) {
    const int p = bi * 32 + r, q = bj * 32 + tx;
    double v = 0.0;
    if (p < M && q < M && p <= q) {
      v = P[packed_row(p, M) + (q - p)];
      F[(size_t)p * M + q] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int q = bj * 32 + r, p = bi * 32 + tx;  // write (q, p) from element (p, q)
    if (p < M && q < M && p < q) F[(size_t)q * M + p] = tile[tx][r];
  }
}

// Synthetic Cholesky vectors by counters (the input recipe documented with
// afqmc_system_desc): every element from four SplitMix64 outputs, so the
// tensor needs no host memory and equals its host twin bit for bit.
__global__ void k_gen_chol(double *__restrict__ L, int M, unsigned long long seed, const double *__restrict__ fac,
                           double root3) {
  const int p = blockIdx.x, g = blockIdx.y;
  const unsigned long long golden = 0x9E3779B97F4A7C15ull;
  for (int q = p + threadIdx.x; q < M; q += blockDim.x) {
    const unsigned long long i = ((unsigned long long)g * M + p) * M + q;
    double u[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      unsigned long long z = seed + (4 * i + r + 1) * golden;
      z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
      z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
      z ^= z >> 31;
      u[r] = (double)(z >> 11) * 0x1p-53;
    }
    const double zsum = ((u[0] + u[1]) + u[2]) + u[3] - 2.0;
    const double v = (zsum * root3) * fac[g];
    L[((size_t)g * M + p) * M + q] = v;
    L[((size_t)g * M + q) * M + p] = v;
  }
}

hipError_t launch_gen_chol(const System &s, uint64_t seed, const double *fac, double root3, hipStream_t st) {
  hipLaunchKernelGGL(k_gen_chol, dim3(s.M, s.G), dim3(kThreads), 0, st, s.L, s.M, (unsigned long long)seed, fac,
                     root3);
  return hipGetLastError();
}

hipError_t launch_pack_upper(const System &s, hipStream_t st) {
  hipLaunchKernelGGL(k_pack_upper, dim3(s.M, s.G), dim3(kThreads), 0, st, s.L, s.M, s.Lp);
  return hipGetLastError();
}

hipError_t launch_vhs(const System &s, int W, hipStream_t st, bool imag_only) {
  if (s.prop32 && s.Lp32) return launch_vhs_f32(s, W, st, imag_only);
  const long MM = (long)s.M * s.M;
  // rows (w, c) of yp; with imag_only the rows (w, 1) alone, into planes (w, 1)
  const int rows = imag_only ? W : 2 * W, rstride = imag_only ? 2 : 1, roff = imag_only ? 1 : 0;
  GemmArgs a;
  a.m = rows; a.k = s.G;
  a.A = s.yp + (size_t)roff * s.G; a.sai = (long)rstride * s.G; a.sak = 1;
  if (s.use_mfma_gemm && s.Lp) {
    const long Mp = (long)s.M * (s.M + 1) / 2;
    a.n = (int)Mp;
    a.B = s.Lp; a.sbk = Mp; a.sbj = 1;
    a.C = s.vhsp + (size_t)roff * Mp; a.sci = rstride * Mp; a.scj = 1;
    hipError_t e = gemm_vhs_mfma(a, st, s.vhs_shape);
    if (e != hipSuccess) return e;
    if (s.prop32) return launch_unpack_f32(s, W, st, imag_only);
    const int nt = (s.M + 31) / 32;
    hipLaunchKernelGGL(k_unpack_symmetric, dim3(nt * (nt + 1) / 2, rows), dim3(kThreads), 0, st, s.vhsp, s.M, nt,
                       rstride, roff, s.vhs);
    return hipGetLastError();
  }
  a.n = (int)MM;
  a.B = s.L; a.sbk = MM; a.sbj = 1;
  a.C = s.vhs + (size_t)roff * MM; a.sci = rstride * MM; a.scj = 1;
  return s.use_mfma_gemm ? gemm_vhs_mfma(a, st, s.vhs_shape) : gemm_f64(a, st);
}

// ---- one-body half step: out_w = B1 in_w (complex columns as real pairs) -----
hipError_t launch_b1(const System &s, const double2 *in, double2 *out, int W, hipStream_t st) {
  const long n2 = 2L * s.Nt;
  GemmArgs a;
  a.m = s.M; a.n = (int)n2; a.k = s.M; a.batch = W;
  a.A = s.B1; a.sai = s.M; a.sak = 1; a.sab = 0;
  a.B = reinterpret_cast<const double *>(in); a.sbk = n2; a.sbj = 1; a.sbb = (long)s.M * n2;
  a.C = reinterpret_cast<double *>(out); a.sci = n2; a.scj = 1; a.scb = (long)s.M * n2;
  return s.use_mfma_gemm ? gemm_b1_mfma(a, st) : gemm_f64(a, st);
}

// ---- Taylor term: tout = alpha (Ar + i Ai) tin, tacc += tout -----------------
// Tile: 64 rows x 16 complex columns per workgroup; each thread owns 4 rows of
// one column.  Ar/Ai rows are contiguous in the contraction index.
__global__ __launch_bounds__(kThreads) void k_taylor_term(const double *__restrict__ vhs,
                                                         const double2 *__restrict__ tin,
                                                         double2 *__restrict__ tout,
                                                         double2 *__restrict__ tacc, int M, int Nt,
                                                         double alpha) {
  __shared__ double Ar[TBK][TBM + 4];
  __shared__ double Ai[TBK][TBM + 4];
  __shared__ double2 Ts[TBK][16];
  const int tid = threadIdx.x, tx = tid & 15, ty = tid >> 4;
  const int j0 = blockIdx.x * 16, i0 = blockIdx.y * TBM, w = blockIdx.z;
  const size_t MM = (size_t)M * M;
  const double *ar = vhs + (size_t)w * 2 * MM;
  const double *ai = ar + MM;
  const double2 *t = tin + (size_t)w * M * Nt;
  double re[4] = {0, 0, 0, 0}, im[4] = {0, 0, 0, 0};
  for (int k0 = 0; k0 < M; k0 += TBK) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int kk = tid & 15, ii = (tid >> 4) + 16 * r;
      const int gi = i0 + ii, gk = k0 + kk;
      const bool ok = gi < M && gk < M;
      Ar[kk][ii] = ok ? ar[(size_t)gi * M + gk] : 0.0;
      Ai[kk][ii] = ok ? ai[(size_t)gi * M + gk] : 0.0;
    }
    {
      const int kk = tid >> 4, jj = tid & 15;
      const int gk = k0 + kk, gj = j0 + jj;
      Ts[kk][jj] = (gk < M && gj < Nt) ? t[(size_t)gk * Nt + gj] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll
    for (int kk = 0; kk < TBK; ++kk) {
      const double2 b = Ts[kk][tx];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double xr = Ar[kk][ty * 4 + r], xi = Ai[kk][ty * 4 + r];
        re[r] = fma(xr, b.x, fma(-xi, b.y, re[r]));
        im[r] = fma(xr, b.y, fma(xi, b.x, im[r]));
      }
    }
    __syncthreads();
  }
  const int gj = j0 + tx;
  if (gj >= Nt) return;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int gi = i0 + ty * 4 + r;
    if (gi >= M) continue;
    const size_t e = (size_t)w * M * Nt + (size_t)gi * Nt + gj;
    const double2 v = make_double2(alpha * re[r], alpha * im[r]);
    tout[e] = v;
    tacc[e] = cadd(tacc[e], v);
  }
}

bool free_half_supported(const System &s) {
  if (s.free_full || !s.use_mfma_gemm) return false;
  return s.prop32 || (s.taylor_kernel && taylor_mfma_supported(s.M, s.Nt));
}

hipError_t launch_taylor_term(const System &s, const double2 *tin, double2 *tout, double alpha, int W,
                              hipStream_t st, int kbeg) {
  if (s.use_mfma_gemm && s.taylor_kernel && taylor_mfma_supported(s.M, s.Nt))
    return launch_taylor_mfma(s, tin, tout, alpha, W, st, kbeg);
  if (kbeg != 0) return hipErrorInvalidValue;
  if (s.use_mfma_gemm) {
    // [Re A | Im A] (M x 2M) times [T ; iT] (2M x 2Nt) per walker
    const long n2 = 2L * s.Nt, MM = (long)s.M * s.M;
    GemmArgs a;
    a.m = s.M; a.n = (int)n2; a.k = 2 * s.M; a.batch = W;
    a.A = s.vhs; a.sai = s.M; a.sab = 2 * MM; a.khalf = s.M; a.aplane = MM;
    a.B = reinterpret_cast<const double *>(tin); a.sbk = n2; a.sbb = (long)s.M * n2;
    a.C = reinterpret_cast<double *>(tout); a.sci = n2; a.scj = 1; a.scb = (long)s.M * n2;
    a.C2 = reinterpret_cast<double *>(s.tacc);
    a.alpha = alpha;
    return gemm_taylor_mfma(a, st);
  }
  dim3 grid((s.Nt + 15) / 16, (s.M + TBM - 1) / TBM, W);
  hipLaunchKernelGGL(k_taylor_term, grid, dim3(kThreads), 0, st, s.vhs, tin, tout, s.tacc, s.M, s.Nt,
                     alpha);
  return hipGetLastError();
}

}  // namespace afqmc
