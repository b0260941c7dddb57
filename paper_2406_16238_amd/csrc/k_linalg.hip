// Overlap, log-determinant and Green's-function factor of every walker, and the
// modified Gram-Schmidt re-orthogonalisation.  FP64 throughout.
//
// Overlap (Sec. 2, eq. ovlp_ratio and the walker expansion): for each spin block
// O_s = Psi_s^T phi_s (N_s x N_s), <Psi_T|phi> = prod_s det O_s, and the mixed
// Green's function G^s_pq = <a+_p a_q> = sum_i Psi_pi Theta_qi with
// Theta_s = phi_s O_s^-1.  One workgroup per walker holds O_s in LDS and inverts
// it in place by Gauss-Jordan elimination with partial (row) pivoting; the
// pivots give the determinant.  The two spin blocks of a walker run in separate
// workgroups; a second small kernel adds their log-determinants.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int OKQ = 32;                                   // rows of phi / Psi staged per pass
constexpr int OBI = 2, OBJ = 4;                           // O entries per thread block: rows x columns
constexpr int OBLK = ((kMaxSpinOrbitals + OBI - 1) / OBI * ((kMaxSpinOrbitals + OBJ - 1) / OBJ) + kThreads - 1) /
                     kThreads;                             // O blocks per thread
constexpr int TBQ = 2, TBJ = 4;                           // Theta entries per thread block: rows x columns
}  // namespace

// One workgroup per (walker, spin block).  LDS: O (N x N complex, inverted in
// place), plus staging for OKQ rows of Psi_s (real) and phi_s (complex).
// part[w][s] = (log |det O_s|, sum of pivot phases, not reduced), spart[w][s] = 1
// when O_s is singular (then Theta_s is not written).
__global__ __launch_bounds__(kThreads) void k_ovlp_theta(const double2 *__restrict__ phi,
                                                        const double *__restrict__ trial, int M, int Na,
                                                        int Nb, double2 *__restrict__ theta,
                                                        double2 *__restrict__ part,
                                                        uint32_t *__restrict__ spart) {
  extern __shared__ double2 sdyn[];
  __shared__ double2 scol[kMaxSpinOrbitals];
  __shared__ int spiv[kMaxSpinOrbitals];
  __shared__ double2 spivval;
  __shared__ int ssing;

  const int w = blockIdx.x, s = blockIdx.y;
  const int tid = threadIdx.x;
  const int Nt = Na + Nb;
  const int nmax = Na > Nb ? Na : Nb;
  double2 *sA = sdyn;                                        // [N][N]
  double2 *sPh = sdyn + nmax * nmax;                         // [OKQ][N]
  double *sPs = reinterpret_cast<double *>(sPh + OKQ * nmax);  // [OKQ][N]
  const double2 *ph = phi + (size_t)w * M * Nt;
  double lre = 0.0, lim = 0.0;  // log det accumulated by thread 0

  {
    const int N = s ? Nb : Na;
    const int off = s ? Na : 0;
    if (N == 0) {
      if (tid == 0) {
        part[(size_t)w * 2 + s] = make_double2(0.0, 0.0);
        spart[(size_t)w * 2 + s] = 0u;
      }
      return;
    }
    const int NN = N * N;
    // O = Psi_s^T phi_s, OKQ rows at a time through LDS.  Each thread owns
    // blocks of OBI x OBJ entries, so a staged row costs OBI + OBJ LDS reads
    // for OBI OBJ complex updates (indices past N are clamped on read and
    // dropped on write); every entry sums over q in the same order.
    const int nbj = (N + OBJ - 1) / OBJ, nob = ((N + OBI - 1) / OBI) * nbj;
    int oi0[OBLK], oj0[OBLK];
#pragma unroll
    for (int b = 0; b < OBLK; ++b) {
      const int bid = tid + b * kThreads;
      oi0[b] = (bid / nbj) * OBI;
      oj0[b] = (bid - (bid / nbj) * nbj) * OBJ;
    }
    double2 o[OBLK][OBI][OBJ];
#pragma unroll
    for (int b = 0; b < OBLK; ++b)
#pragma unroll
      for (int r = 0; r < OBI; ++r)
#pragma unroll
        for (int c = 0; c < OBJ; ++c) o[b][r][c] = make_double2(0.0, 0.0);
    for (int q0 = 0; q0 < M; q0 += OKQ) {
      const int nq = min(OKQ, M - q0);
      for (int e = tid; e < nq * N; e += blockDim.x) {
        const int qq = e / N, j = e - (e / N) * N;
        sPh[qq * N + j] = ph[(size_t)(q0 + qq) * Nt + off + j];
        sPs[qq * N + j] = trial[(size_t)(q0 + qq) * Nt + off + j];
      }
      __syncthreads();
#pragma unroll
      for (int b = 0; b < OBLK; ++b) {
        if (tid + b * kThreads >= nob) continue;
        int ic[OBI], jc[OBJ];
#pragma unroll
        for (int r = 0; r < OBI; ++r) ic[r] = min(oi0[b] + r, N - 1);
#pragma unroll
        for (int c = 0; c < OBJ; ++c) jc[c] = min(oj0[b] + c, N - 1);
        for (int qq = 0; qq < nq; ++qq) {
          double t[OBI];
          double2 pv[OBJ];
#pragma unroll
          for (int r = 0; r < OBI; ++r) t[r] = sPs[qq * N + ic[r]];
#pragma unroll
          for (int c = 0; c < OBJ; ++c) pv[c] = sPh[qq * N + jc[c]];
#pragma unroll
          for (int r = 0; r < OBI; ++r)
#pragma unroll
            for (int c = 0; c < OBJ; ++c)
              o[b][r][c] = make_double2(fma(t[r], pv[c].x, o[b][r][c].x), fma(t[r], pv[c].y, o[b][r][c].y));
        }
      }
      __syncthreads();
    }
#pragma unroll
    for (int b = 0; b < OBLK; ++b) {
      if (tid + b * kThreads >= nob) continue;
#pragma unroll
      for (int r = 0; r < OBI; ++r)
#pragma unroll
        for (int c = 0; c < OBJ; ++c) {
          const int i = oi0[b] + r, j = oj0[b] + c;
          if (i < N && j < N) sA[i * N + j] = o[b][r][c];
        }
    }
    if (tid == 0) ssing = 0;
    __syncthreads();

    for (int k = 0; k < N; ++k) {
      // pivot: largest |A_ik| for i >= k (first index on ties), found by wave 0
      // (the arg-max over its lanes by DPP steps lands in lane 63)
      if (tid < 64) {
        double best = -1.0;
        int bi = k;
        for (int i = k + tid; i < N; i += 64) {
          const double a = cabs2(sA[i * N + k]);
          if (a > best) { best = a; bi = i; }
        }
        wave_argmax_dpp(best, bi);
        if (tid == 63) {
          spiv[k] = bi;
          const double2 pv = sA[bi * N + k];
          spivval = pv;
          if (!(cabs2(pv) > 0.0) || !isfinite(pv.x) || !isfinite(pv.y)) ssing = 1;
        }
      }
      __syncthreads();
      if (ssing) break;
      const int p = spiv[k];
      const double2 pv = spivval;
      if (p != k) {
        for (int j = tid; j < N; j += blockDim.x) {
          const double2 a = sA[k * N + j];
          sA[k * N + j] = sA[p * N + j];
          sA[p * N + j] = a;
        }
      }
      if (tid == 0) {
        lre += 0.5 * log(cabs2(pv));
        lim += atan2(pv.y, pv.x) + (p != k ? 3.14159265358979323846 : 0.0);
      }
      __syncthreads();
      // save column k of the other rows, then scale the pivot row (the pivot
      // position becomes 1 / pivot); the two touch disjoint entries
      const double2 inv = cdiv(make_double2(1.0, 0.0), pv);
      for (int i = tid; i < N; i += blockDim.x)
        if (i != k) scol[i] = sA[i * N + k];
      for (int j = tid; j < N; j += blockDim.x) {
        const double2 a = (j == k) ? make_double2(1.0, 0.0) : sA[k * N + j];
        sA[k * N + j] = cmul(a, inv);
      }
      __syncthreads();
      // eliminate column k from every other row
      for (int e = tid; e < NN; e += blockDim.x) {
        const int i = e / N, j = e - (e / N) * N;
        if (i == k) continue;
        const double2 a = (j == k) ? make_double2(0.0, 0.0) : sA[e];
        sA[e] = csub(a, cmul(scol[i], sA[k * N + j]));
      }
      __syncthreads();
    }
    if (ssing) {
      if (tid == 0) {
        part[(size_t)w * 2 + s] = make_double2(0.0, 0.0);
        spart[(size_t)w * 2 + s] = 1u;
      }
      return;
    }
    // undo the row interchanges as column interchanges, last first
    for (int k = N - 1; k >= 0; --k) {
      const int p = spiv[k];
      if (p != k) {
        for (int i = tid; i < N; i += blockDim.x) {
          const double2 a = sA[i * N + k];
          sA[i * N + k] = sA[i * N + p];
          sA[i * N + p] = a;
        }
      }
      __syncthreads();
    }
    // Theta_s = phi_s O_s^-1, OKQ rows of phi_s at a time through LDS; each
    // thread owns TBQ rows x TBJ columns, every entry summed over k in order
    if (theta) {
      double2 *th = theta + (size_t)w * M * Nt;
      const int tnbj = (N + TBJ - 1) / TBJ;
      for (int q0 = 0; q0 < M; q0 += OKQ) {
        const int nq = min(OKQ, M - q0);
        for (int e = tid; e < nq * N; e += blockDim.x) {
          const int qq = e / N, j = e - (e / N) * N;
          sPh[qq * N + j] = ph[(size_t)(q0 + qq) * Nt + off + j];
        }
        __syncthreads();
        const int tnb = ((nq + TBQ - 1) / TBQ) * tnbj;
        for (int bid = tid; bid < tnb; bid += blockDim.x) {
          const int qb = (bid / tnbj) * TBQ, jb = (bid - (bid / tnbj) * tnbj) * TBJ;
          int qc[TBQ], jc[TBJ];
#pragma unroll
          for (int r = 0; r < TBQ; ++r) qc[r] = min(qb + r, nq - 1);
#pragma unroll
          for (int c = 0; c < TBJ; ++c) jc[c] = min(jb + c, N - 1);
          double re[TBQ][TBJ], im[TBQ][TBJ];
#pragma unroll
          for (int r = 0; r < TBQ; ++r)
#pragma unroll
            for (int c = 0; c < TBJ; ++c) re[r][c] = im[r][c] = 0.0;
          for (int k = 0; k < N; ++k) {
            double2 pv[TBQ], xv[TBJ];
#pragma unroll
            for (int r = 0; r < TBQ; ++r) pv[r] = sPh[qc[r] * N + k];
#pragma unroll
            for (int c = 0; c < TBJ; ++c) xv[c] = sA[k * N + jc[c]];
#pragma unroll
            for (int r = 0; r < TBQ; ++r)
#pragma unroll
              for (int c = 0; c < TBJ; ++c) {
                re[r][c] += pv[r].x * xv[c].x - pv[r].y * xv[c].y;
                im[r][c] += pv[r].x * xv[c].y + pv[r].y * xv[c].x;
              }
          }
#pragma unroll
          for (int r = 0; r < TBQ; ++r)
#pragma unroll
            for (int c = 0; c < TBJ; ++c)
              if (qb + r < nq && jb + c < N)
                th[(size_t)(q0 + qb + r) * Nt + off + jb + c] = make_double2(re[r][c], im[r][c]);
        }
        __syncthreads();
      }
    }
  }
  if (tid == 0) {
    part[(size_t)w * 2 + s] = make_double2(lre, lim);
    spart[(size_t)w * 2 + s] = 0u;
  }
}

// log<Psi_T|phi> = sum of the two spin blocks' log-determinants (phase reduced
// to (-pi, pi]); a walker with a singular block gets log-overlap 0 and the
// singular flag.
__global__ void k_ovlp_finish(const double2 *__restrict__ part, const uint32_t *__restrict__ spart, int W,
                              double2 *__restrict__ logo, uint32_t *__restrict__ stat,
                              uint32_t *__restrict__ flags_or) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const bool singular = (spart[2 * w] | spart[2 * w + 1]) != 0u;
  const double2 a = part[2 * w], b = part[2 * w + 1];
  logo[w] = singular ? make_double2(0.0, 0.0) : make_double2(a.x + b.x, wrap_phase(a.y + b.y));
  if (stat) stat[w] = singular ? (uint32_t)AFQMC_W_SINGULAR : 0u;
  if (flags_or && singular) flags_or[w] |= AFQMC_W_SINGULAR;
}

// Theta of a walker with a singular block is all zero.
__global__ __launch_bounds__(kThreads) void k_theta_zero_singular(const uint32_t *__restrict__ spart, long per,
                                                                 double2 *__restrict__ theta) {
  const int w = blockIdx.x;
  if (!(spart[2 * w] | spart[2 * w + 1])) return;
  double2 *th = theta + (size_t)w * per;
  for (long e = threadIdx.x; e < per; e += blockDim.x) th[e] = make_double2(0.0, 0.0);
}

size_t ovlp_lds_bytes(int nmax) {
  return (size_t)nmax * nmax * sizeof(double2) + (size_t)OKQ * nmax * (sizeof(double2) + sizeof(double));
}

hipError_t ovlp_enable_lds(int nmax) {
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_ovlp_theta), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)ovlp_lds_bytes(kMaxSpinOrbitals));
}

hipError_t launch_ovlp_theta(const double2 *phi, const double *trial, int M, int Na, int Nb, int W,
                             double2 *theta, double2 *logo, uint32_t *stat, uint32_t *flags_or, hipStream_t st,
                             double2 *part, uint32_t *spart) {
  const int nmax = Na > Nb ? Na : Nb;
  hipLaunchKernelGGL(k_ovlp_theta, dim3(W, 2), dim3(kThreads), ovlp_lds_bytes(nmax), st, phi, trial, M, Na, Nb, theta,
                     part, spart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_ovlp_finish, dim3((W + 255) / 256), dim3(256), 0, st, part, spart, W, logo, stat, flags_or);
  if ((e = hipGetLastError()) != hipSuccess || !theta) return e;
  hipLaunchKernelGGL(k_theta_zero_singular, dim3(W), dim3(kThreads), 0, st, spart, (long)M * (Na + Nb), theta);
  return hipGetLastError();
}

// Modified Gram-Schmidt of each spin block: for k = 0..N-1, r_kk = |phi_k|,
// phi_k /= r_kk, r_kj = phi_k^H phi_j and phi_j -= r_kj phi_k for j > k.
// One workgroup per walker; wave v handles columns j = k+1+v, k+1+v+4, ...
// One workgroup per (walker, spin block); logr[w][s] = sum_i log R_ii of the block.
__global__ __launch_bounds__(kThreads) void k_mgs(double2 *__restrict__ phi, int M, int Na, int Nb,
                                                 double *__restrict__ logr_out) {
  __shared__ double2 sr[kMaxSpinOrbitals];
  __shared__ double snorm;
  const int w = blockIdx.x, s = blockIdx.y, tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  const int nw = blockDim.x >> 6;
  const int Nt = Na + Nb;
  double2 *ph = phi + (size_t)w * M * Nt;
  double logr = 0.0;
  {
    const int N = s ? Nb : Na;
    const int off = s ? Na : 0;
    for (int k = 0; k < N; ++k) {
      const int ck = off + k;
      if (wid == 0) {
        double a = 0.0;
        for (int q = lane; q < M; q += 64) a += cabs2(ph[(size_t)q * Nt + ck]);
        a = wave_sum(a);
        if (lane == 0) snorm = sqrt(a);
      }
      __syncthreads();
      const double r = snorm;
      const double ir = 1.0 / r;
      for (int q = tid; q < M; q += blockDim.x) {
        const size_t e = (size_t)q * Nt + ck;
        ph[e] = cscale(ph[e], ir);
      }
      if (tid == 0) logr += log(r);
      __syncthreads();
      for (int j = k + 1 + wid; j < N; j += nw) {
        double re = 0.0, im = 0.0;
        for (int q = lane; q < M; q += 64) {
          const double2 a = ph[(size_t)q * Nt + ck];
          const double2 b = ph[(size_t)q * Nt + off + j];
          re += a.x * b.x + a.y * b.y;  // conj(a) b
          im += a.x * b.y - a.y * b.x;
        }
        re = wave_sum(re);
        im = wave_sum(im);
        if (lane == 0) sr[j] = make_double2(re, im);
      }
      __syncthreads();
      const int nrest = N - k - 1;
      for (int e = tid; e < M * nrest; e += blockDim.x) {
        const int q = e / nrest, j = k + 1 + (e - (e / nrest) * nrest);
        const double2 a = ph[(size_t)q * Nt + ck];
        const size_t ej = (size_t)q * Nt + off + j;
        ph[ej] = csub(ph[ej], cmul(sr[j], a));
      }
      __syncthreads();
    }
  }
  if (tid == 0) logr_out[(size_t)w * 2 + s] = logr;
}

// The same modified Gram-Schmidt with the spin block held in registers: one
// workgroup of 512 threads per (walker, spin block), thread q holding row q
// (M <= 512) of the block's NMAX >= N columns (N <= 48: the row fits the
// registers of two waves per SIMD), so phi is read and written once.
// Norms and the dot products of column k with the later columns are summed
// over the rows by DPP steps within each wave (no LDS traffic) and then over
// the eight waves through LDS in a fixed order; the loops over columns are unrolled so
// the row stays in registers.
template <int NMAX>
__global__ __launch_bounds__(512) void k_mgs_reg(double2 *__restrict__ phi, int M, int Na, int Nb,
                                                double *__restrict__ logr_out) {
  __shared__ double2 sdot[8][NMAX];
  const int w = blockIdx.x, s = blockIdx.y, q = threadIdx.x, lane = q & 63, wv = q >> 6;
  const int Nt = Na + Nb, N = s ? Nb : Na, off = s ? Na : 0;
  double2 *row = phi + ((size_t)w * M + q) * Nt + off;
  double2 c[NMAX];
#pragma unroll
  for (int j = 0; j < NMAX; ++j) c[j] = (q < M && j < N) ? row[j] : make_double2(0.0, 0.0);
  double logr = 0.0;
#pragma clang loop unroll(full)
  for (int k = 0; k < NMAX; ++k) {
    if (k >= N) continue;  // uniform in the workgroup
    // |column k|^2
    const double n2 = wave_sum_dpp(cabs2(c[k]));   // valid in lane 63
    if (lane == 63) sdot[wv][0] = make_double2(n2, 0.0);
    __syncthreads();
    double nn = sdot[0][0].x;
#pragma unroll
    for (int v = 1; v < 8; ++v) nn += sdot[v][0].x;
    const double r = sqrt(nn);
    c[k] = cscale(c[k], 1.0 / r);
    logr += log(r);
    __syncthreads();
    // r_kj = sum_q conj(c_qk) c_qj for j > k, then c_j -= r_kj c_k
#pragma clang loop unroll(full)
    for (int j = k + 1; j < NMAX; ++j) {
      const double re = wave_sum_dpp(c[k].x * c[j].x + c[k].y * c[j].y);
      const double im = wave_sum_dpp(c[k].x * c[j].y - c[k].y * c[j].x);
      if (lane == 63) sdot[wv][j] = make_double2(re, im);
    }
    __syncthreads();
#pragma clang loop unroll(full)
    for (int j = k + 1; j < NMAX; ++j) {
      double2 d = sdot[0][j];
#pragma unroll
      for (int v = 1; v < 8; ++v) d = cadd(d, sdot[v][j]);
      c[j] = csub(c[j], cmul(d, c[k]));
    }
    __syncthreads();
  }
  if (q < M) {
#pragma unroll
    for (int j = 0; j < NMAX; ++j)
      if (j < N) row[j] = c[j];
  }
  if (q == 0) logr_out[(size_t)w * 2 + s] = logr;
}

// log<Psi_T|phi> -= sum over both blocks of log R_ii
__global__ void k_mgs_finish(const double *__restrict__ logr, int W, double2 *__restrict__ logo) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w < W) logo[w].x -= logr[2 * w] + logr[2 * w + 1];
}

hipError_t launch_mgs(double2 *phi, int M, int Na, int Nb, int W, double2 *logo, hipStream_t st, double *scratch) {
  const int n = Na > Nb ? Na : Nb;
  if (M <= 512 && n <= 48) {
    const dim3 g(W, 2), b(512);
    if (n <= 8) hipLaunchKernelGGL(k_mgs_reg<8>, g, b, 0, st, phi, M, Na, Nb, scratch);
    else if (n <= 16) hipLaunchKernelGGL(k_mgs_reg<16>, g, b, 0, st, phi, M, Na, Nb, scratch);
    else if (n <= 24) hipLaunchKernelGGL(k_mgs_reg<24>, g, b, 0, st, phi, M, Na, Nb, scratch);
    else if (n <= 32) hipLaunchKernelGGL(k_mgs_reg<32>, g, b, 0, st, phi, M, Na, Nb, scratch);
    else if (n <= 40) hipLaunchKernelGGL(k_mgs_reg<40>, g, b, 0, st, phi, M, Na, Nb, scratch);
    else hipLaunchKernelGGL(k_mgs_reg<48>, g, b, 0, st, phi, M, Na, Nb, scratch);
  } else {
    hipLaunchKernelGGL(k_mgs, dim3(W, 2), dim3(kThreads), 0, st, phi, M, Na, Nb, scratch);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_mgs_finish, dim3((W + 255) / 256), dim3(256), 0, st, scratch, W, logo);
  return hipGetLastError();
}

}  // namespace afqmc
