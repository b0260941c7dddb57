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
// A = the half-rotated vectors (rows (g, i), padded to NR rows per g), B = the
// walkers' Theta with interleaved complex columns (padded to CP per walker).
// A workgroup owns GC whole Cholesky vectors (RT = GC*NR/16 row tiles) and four
// whole walkers (one per wave, CT = CP/16 column tiles), so every T^{g}_w is
// complete inside one wave and the trace needs no other workgroup.  The K loop
// stages 16 contraction rows of A and B in LDS (double-buffered through
// registers) and issues RT*CT v_mfma_f64_16x16x4f64 per 4 rows.
// MFMA lane layout (16x16x4, f64): lane l supplies A[l%16][l/16] and
// B[l/16][l%16]; accumulator item r of lane l is D[l/16 + 4 r][l%16].
typedef double dvec4 __attribute__((ext_vector_type(4)));

namespace {
constexpr int XKC = 16;     // contraction rows per LDS stage
constexpr int XWALK = 4;    // walkers per workgroup (one per wave)
}  // namespace

template <int RT, int CT>
__global__ __launch_bounds__(kThreads) void k_exchange_mfma(const double *__restrict__ LtT,
                                                           const double *__restrict__ theta, int M, int Nt,
                                                           int off, int N, int NR, int GC, int G, int W,
                                                           int stride, int spin, double2 *__restrict__ ekpart) {
  constexpr int ROWS = RT * 16;
  constexpr int CP = CT * 16;
  constexpr int ASZ = XKC * ROWS;            // doubles per A stage
  constexpr int BSZ = XWALK * XKC * CP;      // doubles per B stage
  constexpr int APT = ASZ / kThreads;        // = RT
  constexpr int BPT = BSZ / kThreads;        // = 4 * CT
  extern __shared__ double smem[];
  double *sA = smem;                 // [2][XKC][ROWS]
  double *sB = smem + 2 * ASZ;       // [2][XWALK][XKC][CP]

  const int gb = blockIdx.x, wb = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int g0 = gb * GC, w0 = wb * XWALK;
  const int twoN = 2 * N;
  const size_t wstride = (size_t)M * Nt * 2;  // doubles per walker

  double ra[APT], rb[BPT];
  auto load = [&](int q0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = tid + r * kThreads;
      const int q = e / ROWS, row = e - q * ROWS;
      const int gl = row / NR, i = row - gl * NR;
      const int g = g0 + gl, gq = q0 + q;
      ra[r] = (i < N && g < G && gq < M) ? LtT[((size_t)g * M + gq) * Nt + off + i] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = tid + r * kThreads;
      const int c = e % CP, t = e / CP;
      const int q = t % XKC, wl = t / XKC;
      const int w = w0 + wl, gq = q0 + q;
      rb[r] = (c < twoN && w < W && gq < M) ? theta[(size_t)w * wstride + (size_t)gq * Nt * 2 + 2 * off + c] : 0.0;
    }
  };
  auto store = [&](int buf) {
    double *a = sA + buf * ASZ;
    double *b = sB + buf * BSZ;
#pragma unroll
    for (int r = 0; r < APT; ++r) a[tid + r * kThreads] = ra[r];
#pragma unroll
    for (int r = 0; r < BPT; ++r) b[tid + r * kThreads] = rb[r];
  };

  dvec4 acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = dvec4{0.0, 0.0, 0.0, 0.0};

  const int nchunk = (M + XKC - 1) / XKC;
  load(0);
  store(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * XKC);
    const double *a = sA + buf * ASZ;
    const double *b = sB + buf * BSZ + wv * XKC * CP;
#pragma unroll
    for (int ks = 0; ks < XKC / 4; ++ks) {
      double av[RT], bv[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) av[i] = a[(ks * 4 + lk) * ROWS + i * 16 + lr];
#pragma unroll
      for (int j = 0; j < CT; ++j) bv[j] = b[(ks * 4 + lk) * CP + j * 16 + lr];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  // epilogue: one Cholesky vector at a time, each wave writes its walker's T
  // (N rows x 2N interleaved columns) to its own LDS region and forms
  // sum_ij T_ij T_ji.
  double *sT = smem + (size_t)wv * N * twoN;
  const int w = w0 + wv;
  double pre = 0.0, pim = 0.0;
  for (int gl = 0; gl < GC; ++gl) {
    const int rbase = gl * NR;
#pragma unroll
    for (int i = 0; i < RT; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          const int row = i * 16 + lk + 4 * r - rbase;
          const int col = j * 16 + lr;
          if (row >= 0 && row < N && col < twoN) sT[row * twoN + col] = acc[i][j][r];
        }
    __syncthreads();
    if (g0 + gl < G && w < W) {
      for (int e = lane; e < N * N; e += 64) {
        const int i = e / N, j = e - i * N;
        const double ar = sT[i * twoN + 2 * j], ai = sT[i * twoN + 2 * j + 1];
        const double br = sT[j * twoN + 2 * i], bi = sT[j * twoN + 2 * i + 1];
        pre += ar * br - ai * bi;
        pim += ar * bi + ai * br;
      }
    }
    __syncthreads();
  }
  pre = wave_sum(pre);
  pim = wave_sum(pim);
  if (lane == 0 && w < W) ekpart[((size_t)w * 2 + spin) * stride + gb] = make_double2(-0.5 * pre, -0.5 * pim);
}

namespace {

using ExKernel = void (*)(const double *, const double *, int, int, int, int, int, int, int, int, int, int,
                          double2 *);

template <int RT>
ExKernel pick_ct(int ct) {
  switch (ct) {
    case 1: return k_exchange_mfma<RT, 1>;
    case 2: return k_exchange_mfma<RT, 2>;
    case 3: return k_exchange_mfma<RT, 3>;
    case 4: return k_exchange_mfma<RT, 4>;
    case 5: return k_exchange_mfma<RT, 5>;
    case 6: return k_exchange_mfma<RT, 6>;
    default: return nullptr;
  }
}

ExKernel pick_exchange(int rt, int ct) {
  switch (rt) {
    case 1: return pick_ct<1>(ct);
    case 2: return pick_ct<2>(ct);
    case 3: return pick_ct<3>(ct);
    case 5: return pick_ct<5>(ct);
    default: return nullptr;
  }
}

}  // namespace

ExchangePlan exchange_plan(int N, int G) {
  ExchangePlan p;
  p.N = N;
  if (N <= 0) return p;
  p.NR = ((N + 7) / 8) * 8;
  p.GC = (p.NR % 16 == 0) ? 1 : 2;
  p.RT = p.GC * p.NR / 16;
  p.CT = (2 * N + 15) / 16;
  p.ngb = (G + p.GC - 1) / p.GC;
  const size_t stage = 2ull * (XKC * p.RT * 16 + XWALK * XKC * p.CT * 16) * sizeof(double);
  const size_t epi = (size_t)XWALK * N * 2 * N * sizeof(double);
  p.lds = stage > epi ? stage : epi;
  p.mfma = pick_exchange(p.RT, p.CT) != nullptr && p.lds <= 160 * 1024;
  if (!p.mfma) p.ngb = 0;
  return p;
}

hipError_t launch_exchange(const System &s, const double2 *theta, int W, hipStream_t st) {
  if (s.ex_mfma) {
    for (int spin = 0; spin < 2; ++spin) {
      const ExchangePlan &p = s.ex_plan[spin];
      if (p.N == 0) continue;
      ExKernel k = pick_exchange(p.RT, p.CT);
      dim3 grid(p.ngb, (W + XWALK - 1) / XWALK);
      hipLaunchKernelGGL(k, grid, dim3(kThreads), p.lds, st, s.LtT, reinterpret_cast<const double *>(theta), s.M,
                         s.Nt, spin ? s.Na : 0, p.N, p.NR, p.GC, s.G, W, s.ex_stride, spin, s.ekpart);
      hipError_t e = hipGetLastError();
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  }
  dim3 grid(s.ex_ngb, 2, W);
  hipLaunchKernelGGL(k_exchange_v1, grid, dim3(kThreads), s.ex_lds, st, s.LtT, theta, s.M, s.Na, s.Nb, s.G,
                     s.ex_gb, s.ex_ngb, s.ekpart);
  return hipGetLastError();
}

hipError_t exchange_enable_lds(const System &s) {
  if (!s.ex_mfma) return hipSuccess;
  for (int spin = 0; spin < 2; ++spin) {
    const ExchangePlan &p = s.ex_plan[spin];
    if (p.N == 0) continue;
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pick_exchange(p.RT, p.CT)),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)p.lds);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace afqmc
