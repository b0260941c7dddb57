// Overlap, log-determinant and Green's-function factor of every walker, and the
// modified Gram-Schmidt re-orthogonalisation.  FP64 throughout.
//
// Overlap (Sec. 2, eq. ovlp_ratio and the walker expansion): for each spin block
// O_s = Psi_s^T phi_s (N_s x N_s), <Psi_T|phi> = prod_s det O_s, and the mixed
// Green's function G^s_pq = <a+_p a_q> = sum_i Psi_pi Theta_qi with
// Theta_s = phi_s O_s^-1.  One workgroup per walker and spin block forms O_s on
// the matrix cores, holds it in LDS and inverts it in place by Gauss-Jordan
// elimination with partial (row) pivoting (the pivots give the determinant),
// then forms Theta_s on the matrix cores.  The two spin blocks of a walker run in separate
// workgroups; a second small kernel adds their log-determinants.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

// Both products run on v_mfma_f64_4x4x4_4b_f64 (four 4x4x4 blocks that share
// one 4-row slab of A; lane 16k+4b+i supplies A[i][k], lane 16k+4b+j supplies
// B[k][4b+j], lane 16i+4b+j receives D[i][4b+j]), with operands read straight
// from memory: a slab r and a 16-column group c of C give C[4r + lane/16]
// [16c + lane%16].  Complex matrices enter as real ones with interleaved
// (re, im) columns.  The kernels are instantiated for NB = ceil(max N / 8):
// O has 2 NB slabs and NB column groups.
// Operands are read through buffer resources: a byte offset past the end of the
// buffer (kOutside) reads zero, so entries outside the matrices need no select
// or branch and a load can be issued steps before its use.
constexpr int kOutside = 0x40000000;   // above every buffer here, and room to add a row offset
__device__ __forceinline__ __amdgpu_buffer_rsrc_t rsrc_of(const void *p, uint32_t bytes) {
  return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(p), 0, bytes, 0x00020000);
}
__device__ __forceinline__ double ld_f64(__amdgpu_buffer_rsrc_t r, int byte_off) {
  return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, byte_off, 0, 0));
}
__device__ __forceinline__ double mfma_f64(double a, double b, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(a, b, c, 0, 0, 0);
}

// One workgroup per (walker, spin block).  LDS: O (N x N complex, inverted in
// place), then B of the Theta product.
// part[w][s] = (log |det O_s|, sum of pivot phases, not reduced), spart[w][s] = 1
// when O_s is singular (then Theta_s is not written).
template <int NB>
__global__ __launch_bounds__(kThreads) void k_ovlp_theta(const double2 *__restrict__ phi,
                                                        const double *__restrict__ trial, int M, int Na,
                                                        int Nb, double2 *__restrict__ theta,
                                                        double2 *__restrict__ part,
                                                        uint32_t *__restrict__ spart) {
  extern __shared__ double2 sdyn[];
  __shared__ double2 scol[kMaxSpinOrbitals];
  __shared__ double2 spv[kMaxSpinOrbitals];   // pivots, in elimination order
  __shared__ int spiv[kMaxSpinOrbitals];      // pivot rows
  __shared__ int scolof[kMaxSpinOrbitals];    // column order that undoes the interchanges
  __shared__ int ssing;
  __shared__ double2 sdump[64];   // sink for results of elimination slots past the matrix
  constexpr int NW = kThreads / 64;
  static_assert(kMaxSpinOrbitals <= 64 && kMaxSpinOrbitals <= 8 * 7, "one lane per column; NB <= 7");
  // O in column passes of at most 4 groups (registers); Theta in batches of TS slabs
  constexpr int RS = 2 * NB, CPASS = NB <= 5 ? NB : (NB + 1) / 2, TS = NB <= 4 ? 8 : 28 / NB;
  constexpr int PD = NB <= 3 ? 4 : NB == 4 ? 3 : 2;   // contraction steps whose operands are in flight
  constexpr int RW = (8 * NB + NW - 1) / NW;           // rows of O per wave in the elimination

  const int w = blockIdx.x, s = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: loop bounds stay scalar
  const int l4 = lane & 3, lk = lane >> 4, l16 = lane & 15;
  const int Nt = Na + Nb;
  const int nmax = Na > Nb ? Na : Nb;
  double2 *sA = sdyn;                                        // [N][N]
  constexpr int LDB = 16 * NB + 1;                           // row stride of sBx (doubles)
  double *sBx = reinterpret_cast<double *>(sdyn + nmax * nmax);   // [8 ceil(N/4)][LDB]
  const double2 *ph = phi + (size_t)w * M * Nt;
  double lre = 0.0, lim = 0.0;  // log det, summed by thread 0

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
    // O = Psi_s^T phi_s as a real N x 2N product over q: wave v takes the
    // 4-row contraction steps v, v + NW, ..., and the waves' partial sums are
    // added in LDS in wave order (a fixed order).  A[i][q] = Psi[q][i],
    // B[q][2j + t] = (re, im) of phi[q][j]; rows past N and columns past 2N
    // read zero and are dropped.
    // trial [M][Nt] and this walker's phi [M][Nt] (complex) as buffers
    const __amdgpu_buffer_rsrc_t rpsi = rsrc_of(trial, (uint32_t)(M * Nt) * 8u);
    const __amdgpu_buffer_rsrc_t rphi = rsrc_of(ph, (uint32_t)(M * Nt) * 16u);
    const int nsteps = (M + 3) / 4;
    for (int c0 = 0; c0 < NB; c0 += CPASS) {
      double acc[RS][CPASS];
#pragma unroll
      for (int r = 0; r < RS; ++r)
#pragma unroll
        for (int c = 0; c < CPASS; ++c) acc[r][c] = 0.0;
      double av[RS], bv[CPASS];
      // byte offsets within a row (kOutside for rows past N, columns past 2N)
      int aoff[RS], boff[CPASS];
#pragma unroll
      for (int r = 0; r < RS; ++r) {
        const int i = 4 * r + l4;
        aoff[r] = i < N ? 8 * (off + i) : kOutside;
      }
#pragma unroll
      for (int c = 0; c < CPASS; ++c) {
        const int col = 16 * (c0 + c) + l16;
        boff[c] = (c0 + c < NB && col < 2 * N) ? 8 * (2 * off + col) : kOutside;
      }
      // (rows q >= M lie past the end of both buffers)
      auto load = [&](int st, double (&aa)[RS], double (&bb)[CPASS]) {
        const int q = 4 * st + lk;
        const int ra = q * Nt * 8, rb = q * Nt * 16;
#pragma unroll
        for (int r = 0; r < RS; ++r) aa[r] = ld_f64(rpsi, ra + aoff[r]);
#pragma unroll
        for (int c = 0; c < CPASS; ++c) bb[c] = ld_f64(rphi, rb + boff[c]);
      };
      // operands of the wave's next PD steps in flight (a rotating set of
      // buffers, indexed statically in the unrolled loop; zero past the end)
      double ab[PD][RS], bb[PD][CPASS];
#pragma unroll
      for (int u = 0; u < PD; ++u) load(wv + NW * u, ab[u], bb[u]);
      const int nst = (nsteps - wv + NW - 1) / NW;
      for (int n0 = 0; n0 < nst; n0 += PD) {
#pragma unroll
        for (int u = 0; u < PD; ++u) {
          if (n0 + u < nst) {
#pragma unroll
            for (int r = 0; r < RS; ++r) av[r] = ab[u][r];
#pragma unroll
            for (int c = 0; c < CPASS; ++c) bv[c] = bb[u][c];
            load(wv + NW * (n0 + u + PD), ab[u], bb[u]);
#pragma unroll
            for (int r = 0; r < RS; ++r)
#pragma unroll
              for (int c = 0; c < CPASS; ++c) acc[r][c] = mfma_f64(av[r], bv[c], acc[r][c]);
          }
        }
      }
      for (int v = 0; v < NW; ++v) {
        if (wv == v) {
#pragma unroll
          for (int r = 0; r < RS; ++r)
#pragma unroll
            for (int c = 0; c < CPASS; ++c) {
              const int i = 4 * r + lk, col = 16 * (c0 + c) + l16;
              if (i < N && c0 + c < NB && col < 2 * N) {
                double *d = reinterpret_cast<double *>(sA + i * N + (col >> 1)) + (col & 1);
                *d = v == 0 ? acc[r][c] : *d + acc[r][c];
              }
            }
        }
        __syncthreads();
      }
    }
    // Gauss-Jordan with partial pivoting.  The pivot of column k is the
    // largest |A_ik| over rows i >= k (first index on ties), found by wave 0
    // (DPP arg-max, result in lane 63).  Each step takes two passes: (1) row k
    // becomes old row p scaled by 1 / pivot (the pivot position 1 / pivot), row
    // p becomes old row k, and scol keeps column k of every other row after
    // the interchange; (2) column k is eliminated from every other row, and
    // wave 0 first updates column k + 1 of all rows and finds the next pivot
    // from those values (the others leave column k + 1 to it).
    auto bad = [](double2 v) { return !(cabs2(v) > 0.0) || !isfinite(v.x) || !isfinite(v.y); };
    auto lane_value = [](double2 v, int src) {   // v of lane src (uniform)
      const long long x = __double_as_longlong(v.x), y = __double_as_longlong(v.y);
      const int xl = __builtin_amdgcn_readlane((int)x, src), xh = __builtin_amdgcn_readlane((int)(x >> 32), src);
      const int yl = __builtin_amdgcn_readlane((int)y, src), yh = __builtin_amdgcn_readlane((int)(y >> 32), src);
      return make_double2(__longlong_as_double(((long long)xh << 32) | (unsigned int)xl),
                          __longlong_as_double(((long long)yh << 32) | (unsigned int)yl));
    };
    if (wv == 0) {
      double best = -1.0;
      int bi = 0;
      double2 a0 = make_double2(0.0, 0.0);
      if (lane < N) {
        a0 = sA[lane * N];
        best = cabs2(a0);
        bi = lane;
      }
      wave_argmax_dpp(best, bi);
      const int p0 = __builtin_amdgcn_readlane(bi, 63);
      const double2 pv0 = lane_value(a0, p0);
      if (lane == 0) {
        spiv[0] = p0;
        spv[0] = pv0;
        ssing = bad(pv0) ? 1 : 0;
      }
    }
    __syncthreads();
    for (int k = 0; k < N; ++k) {
      if (ssing) break;
      const int p = spiv[k];
      // pass 1: wave 0 lane j owns entry j of rows k and p, wave 1 lane i entry i of column k
      if (wv == 0 && lane < N) {
        const int j = lane;
        const double2 inv = cdiv(make_double2(1.0, 0.0), spv[k]);
        const double2 ak = sA[k * N + j], ap = sA[p * N + j];
        if (p != k) sA[p * N + j] = ak;
        sA[k * N + j] = cmul((j == k) ? make_double2(1.0, 0.0) : ap, inv);
        if (j == k && p != k) scol[p] = ak;
      }
      if (wv == 1 && lane < N && lane != k && lane != p) scol[lane] = sA[lane * N + k];
      __syncthreads();
      // pass 2
      const int k1 = k + 1;
      if (wv == 0 && k1 < N) {
        const double2 r1 = sA[k * N + k1];
        double best = -1.0;
        int bi = k1;
        double2 a1 = make_double2(0.0, 0.0);
        if (lane < N && lane != k) {
          a1 = csub(sA[lane * N + k1], cmul(scol[lane], r1));
          sA[lane * N + k1] = a1;
          if (lane >= k1) {
            best = cabs2(a1);
            bi = lane;
          }
        }
        wave_argmax_dpp(best, bi);
        const int p1 = __builtin_amdgcn_readlane(bi, 63);
        const double2 pv1 = lane_value(a1, p1);
        if (lane == 0) {
          spiv[k1] = p1;
          spv[k1] = pv1;
          if (bad(pv1)) ssing = 1;
        }
      }
      // lane j of wave v: column j (not k + 1) of rows v, v + NW, ...; the
      // multiplier scol[i] is one address for the whole wave
      // (all the wave's reads first, from clamped rows; a result that belongs
      // to no entry goes to this lane's slot of sdump)
      if (lane < N && lane != k1) {
        const int j = lane;
        const double2 rk = sA[k * N + j];
        double2 av[RW], cv[RW];
#pragma unroll
        for (int t = 0; t < RW; ++t) {
          const int i = min(wv + NW * t, N - 1);
          av[t] = sA[i * N + j];
          cv[t] = scol[i];
        }
#pragma unroll
        for (int t = 0; t < RW; ++t) {
          const int i = wv + NW * t;
          const double2 a = (j == k) ? make_double2(0.0, 0.0) : av[t];
          double2 *dst = (i < N && i != k) ? sA + i * N + j : sdump + lane;
          *dst = csub(a, cmul(cv[t], rk));
        }
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
    // log det O_s from the pivots: thread i takes log |pivot i| and its phase
    // (plus pi for an interchange), thread 0 sums them in elimination order
    if (tid < N) {
      const double2 pv = spv[tid];
      scol[tid] = make_double2(0.5 * log(cabs2(pv)), atan2(pv.y, pv.x) + (spiv[tid] != tid ? 3.14159265358979323846 : 0.0));
    }
    for (int c = tid; c < N; c += blockDim.x) scolof[c] = c;
    __syncthreads();
    if (tid == 0) {
      for (int k = 0; k < N; ++k) {
        lre += scol[k].x;
        lim += scol[k].y;
      }
      // the row interchanges undone as column interchanges, last first, composed
      // into one order: column c of O_s^-1 is column scolof[c] of sA (the
      // product below reads it so)
      for (int k = N - 1; k >= 0; --k) {
        const int p = spiv[k], t = scolof[k];
        scolof[k] = scolof[p];
        scolof[p] = t;
      }
    }
    __syncthreads();
    // Theta_s = phi_s O_s^-1 as a real M x 2N product over 2N: A = [Re phi |
    // Im phi] (row q), B[k][2j + t] = (Re X, Im X)[k][j] for k < N and
    // (-Im X, Re X)[k - N][j] for k >= N, X = O_s^-1 read through the column
    // order.  Wave v takes 4-row slabs v, v + NW, ... in batches of TS.
    if (theta) {
      double *thr = reinterpret_cast<double *>(theta + (size_t)w * M * Nt + off);
      // contraction steps: the Re half (k < N) then the Im half, ceil(N / 4)
      // each, so which half a step is in is the same for the whole wave
      const int nslab = (M + 3) / 4, khalf = (N + 3) / 4, ksteps = 2 * khalf;
      // B as a real matrix in LDS, rows 4 khalf (Re half) + 4 khalf (Im half),
      // columns 16 NB at stride LDB: B[k][2j + t] = (Re X, Im X)[k][j] and
      // B[4 khalf + k][2j + t] = (-Im X, Re X)[k][j] for k < N, X[k][j] =
      // sA[k][scolof[j]]; zero elsewhere, so the A entries of rows k >= N
      // (finite values of the walker, or past the buffer) add nothing
      const int KR = 8 * khalf;
      for (int e = tid; e < KR * 16 * NB; e += kThreads) {
        const int kk = e / (16 * NB), col = e - kk * (16 * NB);
        const bool hi = kk >= 4 * khalf;
        const int k = hi ? kk - 4 * khalf : kk;
        double v = 0.0;
        if (k < N && col < 2 * N) {
          const double2 x = sA[k * N + scolof[col >> 1]];
          v = hi ? ((col & 1) ? x.x : -x.y) : ((col & 1) ? x.y : x.x);
        }
        sBx[kk * LDB + col] = v;
      }
      __syncthreads();
      for (int sb = wv; sb < nslab; sb += NW * TS) {
        double acc[TS][NB];
#pragma unroll
        for (int r = 0; r < TS; ++r)
#pragma unroll
          for (int c = 0; c < NB; ++c) acc[r][c] = 0.0;
        double av[TS];
        // A entries: row q of slab sb + NW r, contraction index k = 4 ks + lk
        // (Re phi[q][k] for k < N, Im phi[q][k - N] after)
        int qoff[TS];
#pragma unroll
        for (int r = 0; r < TS; ++r) {
          const int q = 4 * (sb + NW * r) + l4;
          qoff[r] = q < M ? 16 * (q * Nt + off) : kOutside;
        }
        auto load = [&](int ks, double (&aa)[TS]) {
          const bool hi = ks >= khalf;
          const int ko = 16 * (4 * (hi ? ks - khalf : ks) + lk) + (hi ? 8 : 0);
#pragma unroll
          for (int r = 0; r < TS; ++r) aa[r] = ld_f64(rphi, qoff[r] + ko);
        };
        auto loadb = [&](int ks, double (&bv)[NB]) {
          const double *b = sBx + min(4 * ks + lk, KR - 1) * LDB + l16;
#pragma unroll
          for (int c = 0; c < NB; ++c) bv[c] = b[16 * c];
        };
        // A operands of the next PD steps in flight, B one step ahead
        double ab[PD][TS], bcur[NB], bnxt[NB];
#pragma unroll
        for (int u = 0; u < PD; ++u) load(u, ab[u]);
        loadb(0, bcur);
        for (int k0 = 0; k0 < ksteps; k0 += PD) {
#pragma unroll
          for (int u = 0; u < PD; ++u) {
            const int ks = k0 + u;
            if (ks < ksteps) {
#pragma unroll
              for (int r = 0; r < TS; ++r) av[r] = ab[u][r];
              load(ks + PD, ab[u]);
              loadb(ks + 1, bnxt);
#pragma unroll
              for (int r = 0; r < TS; ++r)
#pragma unroll
                for (int c = 0; c < NB; ++c) acc[r][c] = mfma_f64(av[r], bcur[c], acc[r][c]);
#pragma unroll
              for (int c = 0; c < NB; ++c) bcur[c] = bnxt[c];
            }
          }
        }
#pragma unroll
        for (int r = 0; r < TS; ++r) {
          const int q = 4 * (sb + NW * r) + lk;
#pragma unroll
          for (int c = 0; c < NB; ++c) {
            const int col = 16 * c + l16;
            if (q < M && col < 2 * N) thr[2 * (size_t)q * Nt + col] = acc[r][c];
          }
        }
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

// O, then the real B matrix of the Theta product
size_t ovlp_lds_bytes(int nmax) {
  const size_t nb = (nmax + 7) / 8, khalf = (nmax + 3) / 4;
  return (size_t)nmax * nmax * sizeof(double2) + 8 * khalf * (16 * nb + 1) * sizeof(double);
}

namespace {
using OvlpKernel = void (*)(const double2 *, const double *, int, int, int, double2 *, double2 *, uint32_t *);
OvlpKernel pick_ovlp(int nmax) {
  switch ((nmax + 7) / 8) {
    case 1: return k_ovlp_theta<1>;
    case 2: return k_ovlp_theta<2>;
    case 3: return k_ovlp_theta<3>;
    case 4: return k_ovlp_theta<4>;
    case 5: return k_ovlp_theta<5>;
    case 6: return k_ovlp_theta<6>;
    default: return k_ovlp_theta<7>;
  }
}
}  // namespace

hipError_t ovlp_enable_lds(int) {
  for (int nb = 1; nb <= 7; ++nb) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(pick_ovlp(8 * nb)),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)ovlp_lds_bytes(8 * nb));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t launch_ovlp_theta(const double2 *phi, const double *trial, int M, int Na, int Nb, int W,
                             double2 *theta, double2 *logo, uint32_t *stat, uint32_t *flags_or, hipStream_t st,
                             double2 *part, uint32_t *spart) {
  const int nmax = Na > Nb ? Na : Nb;
  if (nmax > kMaxSpinOrbitals) return hipErrorInvalidValue;
  hipLaunchKernelGGL(pick_ovlp(nmax), dim3(W, 2), dim3(kThreads), ovlp_lds_bytes(nmax), st, phi, trial, M, Na, Nb,
                     theta, part, spart);
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
