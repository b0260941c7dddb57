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

hipError_t launch_exchange(const System &s, const double2 *theta, int W, hipStream_t st) {
  dim3 grid(s.ex_ngb, 2, W);
  hipLaunchKernelGGL(k_exchange_v1, grid, dim3(kThreads), s.ex_lds, st, s.LtT, theta, s.M, s.Na, s.Nb, s.G,
                     s.ex_gb, s.ex_ngb, s.ekpart);
  return hipGetLastError();
}

}  // namespace afqmc
