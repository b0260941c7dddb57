// FP32 propagation (the paper's mixed-precision variant, Sec. 6: the
// propagation in single precision, energies in double): V_HS stored as FP32
// planes and the Taylor terms of exp(sqrt(dt) V_HS) phi formed in FP32 on
// v_mfma_f32_16x16x4f32, while the series is accumulated, B1 applied and
// everything else computed in FP64.
//
// f32 16x16x4 lane layout: lane l supplies A[l % 16][l / 16] and
// B[l / 16][l % 16], accumulator item r of lane l is D[4 (l / 16) + r][l % 16].
// The contraction is staged 16 indices at a time in LDS (k-major) with 16-byte
// global loads, double-buffered through registers.  M must be a multiple of 4
// (16-byte loads of A never straddle the planes); Nt at most 96.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

typedef float f4t __attribute__((ext_vector_type(4)));

namespace {
constexpr int QKC = 16;   // contraction indices per LDS stage
}  // namespace

// The FP32 term with three real products (the 3M form of the complex product,
// as in the FP64 kernel): P1 = Ar Tr, P2 = Ai Ti, P3 = (Ar + Ai)(Tr + Ti),
// A T = (P1 - P2) + i (P3 - P1 - P2); IMAG (A = i Ai): P1 = Ai Tr, P2 = Ai Ti,
// A T = -P2 + i P1.  WM waves, each 16 rows of one walker by all 16 TNC >= Nt
// complex columns, so the combination stays in registers.  LDS per stage: the
// A planes k-major and the Tr and Ti planes of 16 contraction indices.
template <int WM, int TNC, bool IMAG>
__global__ __launch_bounds__(64 * WM) void k_taylor3m_f32(const float *__restrict__ A32,
                                                        const float2 *__restrict__ tin, float2 *__restrict__ tout,
                                                        double2 *__restrict__ tacc, int M, int Nt, int W, int nrt,
                                                        float alpha) {
  constexpr int NTH = 64 * WM;
  constexpr int BM = 16 * WM, BNC = 16 * TNC;
  constexpr int NPL = IMAG ? 1 : 2;
  constexpr int LDA = BM + 4, LDB = BNC + 4;
  constexpr int AV = NPL * BM * QKC / 4;            // float4 (4 k) of A per stage
  constexpr int BV = QKC * BNC / 2;                 // float4 (2 complex) of T per stage
  constexpr int APT = (AV + NTH - 1) / NTH, BPT = (BV + NTH - 1) / NTH;
  extern __shared__ float qsm[];
  float *sA = qsm;                          // [2 buf][NPL][QKC][LDA]
  float *sB = qsm + 2 * NPL * QKC * LDA;    // [2 buf][2][QKC][LDB]

  const int ntiles = W * nrt;
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = blockIdx.x & 7, jx = blockIdx.x >> 3;
  const int t = x * per + min(x, rem) + jx;
  const int w = t / nrt, i0 = (t - w * nrt) * BM;

  const size_t MM = (size_t)M * M;
  const float *Aw = A32 + (size_t)w * 2 * MM;
  const float2 *Tw = tin + (size_t)w * M * Nt;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int lr = lane & 15, lk = lane >> 4;

  float4 ra[APT], rb[BPT];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * NTH;                 // (plane, row, k quad)
      const int pr = e / (QKC / 4), kq = e - pr * (QKC / 4);
      const int pl = pr / BM, row = pr - pl * BM;
      const int gi = i0 + row, gk = k0 + 4 * kq;
      ra[r] = (e < AV && gi < M && gk < M)
                  ? *reinterpret_cast<const float4 *>(Aw + (IMAG ? 1 : pl) * MM + (size_t)gi * M + gk)
                  : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = tid + r * NTH;                 // (k, complex column pair)
      const int kk = e / (BNC / 2), jp = e - kk * (BNC / 2);
      const int gk = k0 + kk, j = 2 * jp;
      float4 v = make_float4(0.f, 0.f, 0.f, 0.f);
      if (e < BV && gk < M && j < Nt) {
        const float2 *src = Tw + (size_t)gk * Nt + j;
        const float2 z0 = src[0];
        const float2 z1 = (j + 1 < Nt) ? src[1] : make_float2(0.f, 0.f);
        v = make_float4(z0.x, z0.y, z1.x, z1.y);
      }
      rb[r] = v;
    }
  };
  auto store = [&](int buf) {
    float *a = sA + buf * NPL * QKC * LDA;
    float *b = sB + buf * 2 * QKC * LDB;
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * NTH;
      if (e < AV) {
        const int pr = e / (QKC / 4), kq = e - pr * (QKC / 4);
        const int pl = pr / BM, row = pr - pl * BM;
        float *ap = a + (pl * QKC + 4 * kq) * LDA + row;
        ap[0 * LDA] = ra[r].x;
        ap[1 * LDA] = ra[r].y;
        ap[2 * LDA] = ra[r].z;
        ap[3 * LDA] = ra[r].w;
      }
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = tid + r * NTH;
      if (e < BV) {
        const int kk = e / (BNC / 2), jp = e - kk * (BNC / 2);
        *reinterpret_cast<float2 *>(b + kk * LDB + 2 * jp) = make_float2(rb[r].x, rb[r].z);
        *reinterpret_cast<float2 *>(b + (QKC + kk) * LDB + 2 * jp) = make_float2(rb[r].y, rb[r].w);
      }
    }
  };

  f4t p1[TNC], p2[TNC], p3[TNC];
#pragma unroll
  for (int j = 0; j < TNC; ++j) p1[j] = p2[j] = p3[j] = f4t{0.f, 0.f, 0.f, 0.f};

  const int nchunk = (M + QKC - 1) / QKC;
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * QKC);
    const float *a0 = sA + buf * NPL * QKC * LDA + wv * 16 + lr;
    const float *br = sB + buf * 2 * QKC * LDB + lr;
    const float *bi = br + QKC * LDB;
#pragma unroll
    for (int ks = 0; ks < QKC / 4; ++ks) {
      const int kr = ks * 4 + lk;
      float yr[TNC], yi[TNC];
#pragma unroll
      for (int j = 0; j < TNC; ++j) {
        yr[j] = br[kr * LDB + j * 16];
        yi[j] = bi[kr * LDB + j * 16];
      }
      if constexpr (IMAG) {
        const float xi = a0[kr * LDA];
#pragma unroll
        for (int j = 0; j < TNC; ++j) {
          p1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yr[j], p1[j], 0, 0, 0);
          p2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yi[j], p2[j], 0, 0, 0);
        }
      } else {
        const float xr = a0[kr * LDA], xi = a0[(QKC + kr) * LDA];
#pragma unroll
        for (int j = 0; j < TNC; ++j) {
          p1[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xr, yr[j], p1[j], 0, 0, 0);
          p2[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xi, yi[j], p2[j], 0, 0, 0);
        }
        const float xs = xr + xi;
#pragma unroll
        for (int j = 0; j < TNC; ++j) p3[j] = __builtin_amdgcn_mfma_f32_16x16x4f32(xs, yr[j] + yi[j], p3[j], 0, 0, 0);
      }
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  float2 *to = tout + (size_t)w * M * Nt;
  double2 *ta = tacc + (size_t)w * M * Nt;
#pragma unroll
  for (int j = 0; j < TNC; ++j)
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int gi = i0 + wv * 16 + 4 * lk + r;
      const int c = 16 * j + lr;
      if (gi < M && c < Nt) {
        const size_t off = (size_t)gi * Nt + c;
        const float re = IMAG ? -p2[j][r] : p1[j][r] - p2[j][r];
        const float im = IMAG ? p1[j][r] : (p3[j][r] - p1[j][r]) - p2[j][r];
        const float2 v = make_float2(alpha * re, alpha * im);
        to[off] = v;
        const double2 o = ta[off];
        ta[off] = make_double2(o.x + (double)v.x, o.y + (double)v.y);
      }
    }
}

// out[i] = float(in[i]) for n complex values
__global__ void k_c128_to_c64(const double2 *__restrict__ in, long n, float2 *__restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) out[e] = make_float2((float)in[e].x, (float)in[e].y);
}

// full32[m][p][q] = full32[m][q][p] = float(packed[m][t(p, q)]) for p <= q (as
// the FP64 unpacking, writing FP32 planes)
template <typename P>
__global__ __launch_bounds__(kThreads) void k_unpack_symmetric_f32(const P *__restrict__ packed, long ldp, int M,
                                                                   int ntile, int pstride, int poff,
                                                                   float *__restrict__ full) {
  __shared__ float tile[32][33];
  const int m = blockIdx.y * pstride + poff;
  int t = blockIdx.x, bi = 0;
  while (t >= ntile - bi) {
    t -= ntile - bi;
    ++bi;
  }
  const int bj = bi + t;
  const P *Pm = packed + (size_t)m * ldp;
  float *F = full + (size_t)m * M * M;
  const int tx = threadIdx.x & 31, ty = threadIdx.x >> 5;
  for (int r = ty; r < 32; r += 8) {
    const int p = bi * 32 + r, q = bj * 32 + tx;
    float v = 0.f;
    if (p < M && q < M && p <= q) {
      v = (float)Pm[(long)p * M - (long)p * (p - 1) / 2 + (q - p)];
      F[(size_t)p * M + q] = v;
    }
    tile[r][tx] = v;
  }
  __syncthreads();
  for (int r = ty; r < 32; r += 8) {
    const int q = bj * 32 + r, p = bi * 32 + tx;
    if (p < M && q < M && p < q) F[(size_t)q * M + p] = tile[tx][r];
  }
}

// FP32 propagation: the V_HS product in FP32 as well,
//   C[r][c] = sum_g Y[r][g] Lp32[g][c]  (Y read as FP64 rows and rounded),
// rows r = the field rows (w, re/im) or (w, im), columns the packed upper
// triangle (ldb >= M(M+1)/2, a multiple of 4, zero-padded).  128 x 128 tiles,
// 2 x 2 waves of 64 x 64 on v_mfma_f32_16x16x4f32, 16 contraction indices per
// LDS stage double-buffered through registers; workgroups remapped so that
// each XCD walks a contiguous range of tiles, row tiles fastest.
namespace {
constexpr int VBM = 128, VBN = 128, VKC = 16;
}
__global__ __launch_bounds__(kThreads) void k_vhs_f32(const double *__restrict__ Y, long lda, int R, int K,
                                                     const float *__restrict__ B, long ldb, int N,
                                                     float *__restrict__ C, long ldc, int gx, int gy) {
  constexpr int LDA = VBM + 4, LDB = VBN + 4;
  __shared__ __attribute__((aligned(16))) float sA[2][VKC][LDA];
  __shared__ __attribute__((aligned(16))) float sB[2][VKC][LDB];
  const int nb = gx * gy;
  int lin = blockIdx.x;
  const int per = nb / 8;
  if (lin < per * 8) lin = (lin % 8) * per + lin / 8;
  const int bx = lin % gx, by = lin / gx;
  const int r0 = bx * VBM, c0 = by * VBN;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wm = wv >> 1, wn = wv & 1;
  const int lr = lane & 15, lk = lane >> 4;

  double2 ra[4];
  float4 rb[2];
  auto load = [&](int k0) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * kThreads;             // (row, k pair): 128 x 8
      const int row = e >> 3, kp = e & 7;
      const int gr = r0 + row, gk = k0 + 2 * kp;
      double2 v = make_double2(0.0, 0.0);
      if (gr < R) {
        if (gk + 1 < K) v = make_double2(Y[(size_t)gr * lda + gk], Y[(size_t)gr * lda + gk + 1]);
        else if (gk < K) v.x = Y[(size_t)gr * lda + gk];
      }
      ra[r] = v;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = tid + r * kThreads;             // (k, column quad): 16 x 32
      const int kk = e >> 5, cq = e & 31;
      const int gk = k0 + kk, gc = c0 + 4 * cq;
      rb[r] = (gk < K && gc < ldb) ? *reinterpret_cast<const float4 *>(B + (size_t)gk * ldb + gc)
                                   : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int e = tid + r * kThreads;
      const int row = e >> 3, kp = e & 7;
      sA[buf][2 * kp][row] = (float)ra[r].x;
      sA[buf][2 * kp + 1][row] = (float)ra[r].y;
    }
#pragma unroll
    for (int r = 0; r < 2; ++r) {
      const int e = tid + r * kThreads;
      const int kk = e >> 5, cq = e & 31;
      *reinterpret_cast<float4 *>(&sB[buf][kk][4 * cq]) = rb[r];
    }
  };

  f4t acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4t{0.f, 0.f, 0.f, 0.f};
  const int nchunk = (K + VKC - 1) / VKC;
  load(0);
  store(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * VKC);
#pragma unroll
    for (int ks = 0; ks < VKC / 4; ++ks) {
      const int kk = ks * 4 + lk;
      float av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = sA[buf][kk][wm * 64 + 16 * i + lr];
#pragma unroll
      for (int j = 0; j < 4; ++j) bv[j] = sB[buf][kk][wn * 64 + 16 * j + lr];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int gr = r0 + wm * 64 + 16 * i + 4 * lk + r, gc = c0 + wn * 64 + 16 * j + lr;
        if (gr < R && gc < N) C[(size_t)gr * ldc + gc] = acc[i][j][r];
      }
}

// out[i] = float(in[i]) for a [rows][n] array into [rows][ldo] (pad columns zeroed)
__global__ void k_pack_to_f32(const double *__restrict__ in, long n, long rows, long ldo, float *__restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= rows * ldo) return;
  const long r = e / ldo, c = e - r * ldo;
  out[e] = c < n ? (float)in[r * n + c] : 0.f;
}

hipError_t launch_pack_to_f32(const double *in, long n, long rows, long ldo, float *out, hipStream_t st) {
  const long tot = rows * ldo;
  hipLaunchKernelGGL(k_pack_to_f32, dim3((unsigned)((tot + 255) / 256)), dim3(256), 0, st, in, n, rows, ldo, out);
  return hipGetLastError();
}

hipError_t launch_vhs_f32(const System &s, int W, hipStream_t st, bool imag_only) {
  const long Mp = (long)s.M * (s.M + 1) / 2;
  const int rows = imag_only ? W : 2 * W, rstride = imag_only ? 2 : 1, roff = imag_only ? 1 : 0;
  const int gx = (rows + VBM - 1) / VBM, gy = (int)((Mp + VBN - 1) / VBN);
  float *packed = reinterpret_cast<float *>(s.vhsp);      // [2W][Mp] floats in the FP64 packed buffer
  hipLaunchKernelGGL(k_vhs_f32, dim3((unsigned)(gx * gy)), dim3(kThreads), 0, st, s.yp + (size_t)roff * s.G,
                     (long)rstride * s.G, rows, s.G, s.Lp32, s.ldlp32, (int)Mp, packed + (size_t)roff * Mp,
                     (long)rstride * Mp, gx, gy);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const int nt = (s.M + 31) / 32;
  hipLaunchKernelGGL(k_unpack_symmetric_f32<float>, dim3(nt * (nt + 1) / 2, imag_only ? W : 2 * W), dim3(kThreads),
                     0, st, packed, Mp, s.M, nt, rstride, roff, s.vhs32);
  return hipGetLastError();
}

namespace {
template <int WM, int TNC, bool IMAG>
hipError_t run_taylor3m_f32(const System &s, const float2 *tin, float2 *tout, double alpha, int W, hipStream_t st) {
  constexpr int BM = 16 * WM, BNC = 16 * TNC;
  const size_t lds = 2ull * QKC * ((IMAG ? 1 : 2) * (BM + 4) + 2 * (BNC + 4)) * sizeof(float);
  const int nrt = (s.M + BM - 1) / BM;
  hipLaunchKernelGGL((k_taylor3m_f32<WM, TNC, IMAG>), dim3((unsigned)(W * nrt)), dim3(64 * WM), lds, st, s.vhs32,
                     tin, tout, s.tacc, s.M, s.Nt, W, nrt, (float)alpha);
  return hipGetLastError();
}

template <int WM, bool IMAG>
hipError_t run_taylor3m_f32_tn(const System &s, const float2 *tin, float2 *tout, double alpha, int W,
                               hipStream_t st) {
  switch ((s.Nt + 15) / 16) {
    case 1: return run_taylor3m_f32<WM, 1, IMAG>(s, tin, tout, alpha, W, st);
    case 2: return run_taylor3m_f32<WM, 2, IMAG>(s, tin, tout, alpha, W, st);
    case 3: return run_taylor3m_f32<WM, 3, IMAG>(s, tin, tout, alpha, W, st);
    case 4: return run_taylor3m_f32<WM, 4, IMAG>(s, tin, tout, alpha, W, st);
    case 5: return run_taylor3m_f32<WM, 5, IMAG>(s, tin, tout, alpha, W, st);
    default: return run_taylor3m_f32<WM, 6, IMAG>(s, tin, tout, alpha, W, st);
  }
}
}  // namespace

bool prop32_supported(int M, int Nt) { return M % 4 == 0 && Nt >= 1 && Nt <= 96; }

// shape 0: 48-row tiles, 1: 32 rows, 2: 64 rows (measured at the headline
// shape: 48 rows fastest, the smaller grid tail outweighing the extra re-reads
// of T)
hipError_t launch_taylor_f32(const System &s, const float2 *tin, float2 *tout, double alpha, int W, hipStream_t st,
                             int kbeg) {
  // three real products (two for a purely imaginary V_HS, kbeg = M)
  if (kbeg != 0 && kbeg != s.M) return hipErrorInvalidValue;
  const bool imag = kbeg != 0;
  switch (s.taylor_shape) {
    case 1: return imag ? run_taylor3m_f32_tn<2, true>(s, tin, tout, alpha, W, st)
                        : run_taylor3m_f32_tn<2, false>(s, tin, tout, alpha, W, st);
    case 2: return imag ? run_taylor3m_f32_tn<4, true>(s, tin, tout, alpha, W, st)
                        : run_taylor3m_f32_tn<4, false>(s, tin, tout, alpha, W, st);
    default: return imag ? run_taylor3m_f32_tn<3, true>(s, tin, tout, alpha, W, st)
                         : run_taylor3m_f32_tn<3, false>(s, tin, tout, alpha, W, st);
  }
}

hipError_t launch_c128_to_c64(const double2 *in, long n, float2 *out, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_c128_to_c64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, in, n, out);
  return hipGetLastError();
}

hipError_t launch_unpack_f32(const System &s, int W, hipStream_t st, bool imag_only) {
  const int nt = (s.M + 31) / 32;
  const int pstride = imag_only ? 2 : 1, poff = imag_only ? 1 : 0;
  hipLaunchKernelGGL(k_unpack_symmetric_f32<double>, dim3(nt * (nt + 1) / 2, imag_only ? W : 2 * W), dim3(kThreads),
                     0, st, s.vhsp, (long)s.M * (s.M + 1) / 2, s.M, nt, pstride, poff, s.vhs32);
  return hipGetLastError();
}

}  // namespace afqmc
