// Learned control variate for the exchange energy of the local energy
// (eq. Eloc: E2 = EJ + EK with EK the exchange term).  Per walker a small
// network predicts EK from quantities the step already has; the exact EK is
// computed on a uniform random subset S of k walkers only, and every walker
// gets the Horvitz-Thompson estimate
//   g_w = f_w + [w in S] (EK_w - f_w) / pi,   pi = k / W,
// whose expectation over S is EK_w.
//
// Features (double): Re EJ, Im EJ, Re E1, Im E1, sum_g |vbias_g - l_g|^2,
// Re sum_g (vbias_g - l_g)^2, cos and sin of arg <Psi_T|phi>.
// Network (FP32): x (8, standardised) -> tanh(W1 x + b1) (128)
// -> tanh(W2 h + b2) (128) -> W3 h + b3 (2: standardised Re and Im of EK).
// Parameters, flat: W1 [128][8], b1 [128], W2 [128][128], b2 [128], W3 [2][128], b3 [2].
// Normalisation, double [20]: feature means [8], deviations [8], target means [2],
// deviations [2].
// Training: mean over a minibatch of 1/2 ||y - t||^2, gradients by
// backpropagation (per-workgroup partial sums reduced in a fixed order), Adam
// (beta1 = 0.9, beta2 = 0.999, eps = 1e-8, bias-corrected).
// Subset keys: the SplitMix64 output function of seed + call 2^32 + w phi64
// (phi64 = 0x9E3779B97F4A7C15, the golden-ratio increment); the k walkers with
// the smallest keys (ties to the lower index) form S.
#include <cmath>

#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

namespace {
constexpr int NF = kCvFeatures, NH = kCvHidden, NO = 2;
constexpr int P_W1 = 0, P_B1 = NH * NF, P_W2 = P_B1 + NH, P_B2 = P_W2 + NH * NH, P_W3 = P_B2 + NH,
              P_B3 = P_W3 + NO * NH, NP = P_B3 + NO;
static_assert(NP == kCvParams, "parameter layout");
constexpr int CB = kCvGradBlock;  // samples per workgroup of the network kernels
constexpr int S2 = NH + 1;      // LDS row stride of W2 (odd: conflict-free row and column walks)
constexpr unsigned long long kGolden = 0x9E3779B97F4A7C15ull;

// dynamic LDS of the network kernels: W2, h1, h2, d2, d1 (floats)
constexpr size_t kNetLds = (size_t)(NH * S2 + 4 * CB * S2) * sizeof(float);

__device__ __forceinline__ unsigned long long splitmix64(unsigned long long x) {
  unsigned long long z = x + kGolden;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
  return z ^ (z >> 31);
}
}  // namespace

// ---- features ---------------------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_cv_features(const double2 *__restrict__ part, int nslices, int G,
                                                          int W, const double *__restrict__ lmf,
                                                          const double2 *__restrict__ e1,
                                                          const double2 *__restrict__ ej,
                                                          const double2 *__restrict__ logo,
                                                          const double2 *__restrict__ lin,
                                                          double *__restrict__ feat) {
  __shared__ double red[4 * 2];
  const int w = blockIdx.x, tid = threadIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int g = tid; g < G; g += blockDim.x) {
    double2 vb = make_double2(0.0, 0.0);
    for (int s = 0; s < nslices; ++s) vb = cadd(vb, part[((size_t)s * W + w) * G + g]);
    const double dx = vb.x - lmf[g], dy = vb.y;
    acc[0] += dx * dx + dy * dy;
    acc[1] += dx * dx - dy * dy;
  }
  block_sum<2>(acc, red);
  if (tid == 0) {
    const double2 a = ej[w], b = e1[w];
    const double ph = logo[w].y;
    double *f = feat + (size_t)w * NF;
    f[0] = a.x;
    f[1] = a.y;
    f[2] = b.x;
    f[3] = b.y;
    f[4] = acc[0];
    f[5] = acc[1];
    f[6] = cos(ph);
    f[7] = sin(ph);
    f[8] = lin[w].x;
    f[9] = lin[w].y;
  }
}

// K_s[i][q] = sum_g sum_j T0_g[i][j] Ltilde^{g s}[j][q] for i, j of one spin
// block, T0_g = Ltilde^{g s} Psi_s (in t0 [G][Nt][Nt], the cross-spin blocks
// unused); written as KtT[q][i'] (the layout of the half-rotated h).  One
// thread per (q, i'), the sum over g and j in a fixed order.
__global__ void k_cv_kmat(const double *__restrict__ LtT, const double *__restrict__ t0, int G, int M, int Nt, int Na,
                          double *__restrict__ KtT) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)M * Nt) return;
  const int q = (int)(e / Nt), ip = (int)(e - (e / Nt) * Nt);
  const int j0 = ip < Na ? 0 : Na, j1 = ip < Na ? Na : Nt;
  double a = 0.0;
  for (int g = 0; g < G; ++g) {
    const double *t = t0 + ((size_t)g * Nt + ip) * Nt;
    const double *l = LtT + ((size_t)g * M + q) * Nt;
    for (int j = j0; j < j1; ++j) a = fma(t[j], l[j], a);
  }
  KtT[e] = a;
}

hipError_t launch_cv_kmat(System &s, double *t0, hipStream_t st) {
  // t0[g] = LtT[g]^T trial (Nt x Nt per Cholesky vector)
  GemmArgs g;
  g.m = s.Nt; g.n = s.Nt; g.k = s.M; g.batch = s.G;
  g.A = s.LtT; g.sai = 1; g.sak = s.Nt; g.sab = (long)s.M * s.Nt;
  g.B = s.trial; g.sbk = s.Nt; g.sbj = 1; g.sbb = 0;
  g.C = t0; g.sci = s.Nt; g.scj = 1; g.scb = (long)s.Nt * s.Nt;
  hipError_t e = gemm_f64(g, st);
  if (e != hipSuccess) return e;
  const long n = (long)s.M * s.Nt;
  hipLaunchKernelGGL(k_cv_kmat, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.LtT, t0, s.G, s.M, s.Nt, s.Na,
                     s.KtT);
  return hipGetLastError();
}

// ---- subset draw ------------------------------------------------------------------
// One workgroup of 1024 threads; keys in LDS (W <= kCvMaxWalkers).  sel[0..k) =
// the chosen walkers in increasing order, pos[w] = their index in sel or -1.
// The call counter is read once and advanced by one.
__global__ __launch_bounds__(1024) void k_cv_subset(int W, int k, unsigned long long seed,
                                                    unsigned long long *__restrict__ counter,
                                                    unsigned long long *__restrict__ last_call,
                                                    int *__restrict__ sel, int *__restrict__ pos) {
  __shared__ unsigned long long keys[kCvMaxWalkers];
  __shared__ int cnt[1024];
  const int tid = threadIdx.x;
  const unsigned long long call = counter[0];
  for (int w = tid; w < W; w += 1024) keys[w] = splitmix64(seed + (call << 32) + (unsigned long long)w * kGolden);
  __syncthreads();
  if (tid == 0) {
    counter[0] = call + 1;
    last_call[0] = call;
  }
  const int per = (W + 1023) / 1024;
  const int w0 = tid * per, w1 = min(W, w0 + per);
  int c = 0;
  for (int w = w0; w < w1; ++w) {
    const unsigned long long kw = keys[w];
    int r = 0;
    for (int v = 0; v < W; ++v) {
      const unsigned long long kv = keys[v];
      r += (kv < kw || (kv == kw && v < w)) ? 1 : 0;
    }
    const bool in = r < k;
    pos[w] = in ? 1 : -1;  // marked; offsets below
    c += in ? 1 : 0;
  }
  cnt[tid] = c;
  __syncthreads();
  if (tid == 0) {
    int s = 0;
    for (int t = 0; t < 1024; ++t) {
      const int v = cnt[t];
      cnt[t] = s;
      s += v;
    }
  }
  __syncthreads();
  int o = cnt[tid];
  for (int w = w0; w < w1; ++w) {
    if (pos[w] > 0) {
      sel[o] = w;
      pos[w] = o++;
    }
  }
}

// theta_sub[j] = theta[sel[j]] (whole walkers of [M][Nt] double2)
__global__ void k_cv_gather(const double2 *__restrict__ theta, const int *__restrict__ sel, int k, long per,
                            double2 *__restrict__ out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)k * per) return;
  const long j = e / per, r = e - j * per;
  out[e] = theta[(size_t)sel[j] * per + r];
}

// E = E1 + EJ + g, E2 = EJ + g with g the Horvitz-Thompson exchange estimate.
// ekpart rows are those of the compacted subset (row pos[w]).
__global__ __launch_bounds__(kThreads) void k_cv_combine(const double2 *__restrict__ e1,
                                                         const double2 *__restrict__ ej,
                                                         const double2 *__restrict__ ekpart, int stride, int n0,
                                                         int n1, const double2 *__restrict__ f,
                                                         const int *__restrict__ pos, double inv_pi,
                                                         const uint32_t *__restrict__ stat,
                                                         double2 *__restrict__ e_out) {
  __shared__ double red[4 * 2];
  const int w = blockIdx.x;
  const int j = pos[w];
  double acc[2] = {0.0, 0.0};
  if (j >= 0) {
    const double2 *p = ekpart + (size_t)j * 2 * stride;
    for (int q = threadIdx.x; q < n0; q += blockDim.x) {
      acc[0] += p[q].x;
      acc[1] += p[q].y;
    }
    for (int q = threadIdx.x; q < n1; q += blockDim.x) {
      acc[0] += p[stride + q].x;
      acc[1] += p[stride + q].y;
    }
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    const double2 fw = f[w];
    const double2 g = j >= 0 ? make_double2(fw.x + (acc[0] - fw.x) * inv_pi, fw.y + (acc[1] - fw.y) * inv_pi) : fw;
    const double2 a = e1[w], b = ej[w];
    const double2 e2 = cadd(b, g);
    const bool sing = stat[w] != 0u;
    const double2 z = make_double2(0.0, 0.0);
    e_out[(size_t)w * 3 + 0] = sing ? z : cadd(a, e2);
    e_out[(size_t)w * 3 + 1] = sing ? z : a;
    e_out[(size_t)w * 3 + 2] = sing ? z : e2;
  }
}

// exact EK of every walker from the exchange partials (collection of samples)
__global__ __launch_bounds__(kThreads) void k_cv_ek(const double2 *__restrict__ ekpart, int stride, int n0, int n1,
                                                    double2 *__restrict__ ek) {
  __shared__ double red[4 * 2];
  const int w = blockIdx.x;
  const double2 *p = ekpart + (size_t)w * 2 * stride;
  double acc[2] = {0.0, 0.0};
  for (int q = threadIdx.x; q < n0; q += blockDim.x) {
    acc[0] += p[q].x;
    acc[1] += p[q].y;
  }
  for (int q = threadIdx.x; q < n1; q += blockDim.x) {
    acc[0] += p[stride + q].x;
    acc[1] += p[stride + q].y;
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) ek[w] = make_double2(acc[0], acc[1]);
}

// ---- network --------------------------------------------------------------------
namespace {
// Loads W2 into LDS (row stride S2) and runs the two hidden layers for CB
// samples whose standardised inputs are in sx[CB][NF]; thread j owns unit j.
__device__ __forceinline__ void net_hidden(const float *__restrict__ P, const float (*sx)[NF], float *sW2, float *sh1,
                                           float *sh2) {
  const int j = threadIdx.x;
  for (int e = j; e < NH * NH; e += NH) sW2[(e / NH) * S2 + (e % NH)] = P[P_W2 + e];
  float w1[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) w1[i] = P[P_W1 + j * NF + i];
  const float b1 = P[P_B1 + j], b2 = P[P_B2 + j];
#pragma unroll
  for (int b = 0; b < CB; ++b) {
    float z = b1;
#pragma unroll
    for (int i = 0; i < NF; ++i) z = fmaf(w1[i], sx[b][i], z);
    sh1[b * S2 + j] = tanhf(z);
  }
  __syncthreads();
  const float *row = sW2 + j * S2;
  for (int b = 0; b < CB; ++b) {
    float z = b2;
    const float *h = sh1 + b * S2;
    for (int k = 0; k < NH; ++k) z = fmaf(row[k], h[k], z);
    sh2[b * S2 + j] = tanhf(z);
  }
  __syncthreads();
}

__device__ __forceinline__ float net_out(const float *__restrict__ P, const float *sh2, int b, int o) {
  float z = P[P_B3 + o];
  const float *h = sh2 + b * S2;
  for (int k = 0; k < NH; ++k) z = fmaf(P[P_W3 + o * NH + k], h[k], z);
  return z;
}
}  // namespace

// f[s] = prediction of EK for raw features feat[s] (double), s < n.
__global__ __launch_bounds__(NH) void k_cv_predict(const float *__restrict__ P, const double *__restrict__ norm,
                                                   const double *__restrict__ feat, int n,
                                                   double2 *__restrict__ f) {
  extern __shared__ float nsm[];
  __shared__ float sx[CB][NF];
  float *sW2 = nsm, *sh1 = nsm + NH * S2, *sh2 = sh1 + CB * S2;
  const int n0 = blockIdx.x * CB, tid = threadIdx.x;
  for (int e = tid; e < CB * NF; e += NH) {
    const int b = e / NF, i = e % NF, s = n0 + b;
    sx[b][i] = s < n ? (float)((feat[(size_t)s * NF + i] - norm[i]) / norm[NF + i]) : 0.f;
  }
  __syncthreads();
  net_hidden(P, sx, sW2, sh1, sh2);
  if (tid < CB * NO) {
    const int b = tid / NO, o = tid % NO, s = n0 + b;
    const float y = net_out(P, sh2, b, o);
    if (s < n) {
      const double v = (double)y * norm[2 * NF + NO + o] + norm[2 * NF + o];
      reinterpret_cast<double *>(f)[(size_t)s * 2 + o] = v;
    }
  }
}

// Loss and gradient partial sums of samples [n0, n0 + nb) of standardised
// inputs X [n][8] and targets T [n][2]; this workgroup takes CB of them.
// part[wg][NP], lpart[wg]; inv_n = 1 / nb.
__global__ __launch_bounds__(NH) void k_cv_grad(const float *__restrict__ P, const float *__restrict__ X,
                                                const float *__restrict__ T, int n0, int nb, float inv_n,
                                                float *__restrict__ part, double *__restrict__ lpart) {
  extern __shared__ float nsm[];
  __shared__ float sx[CB][NF];
  __shared__ float sr[CB][NO];
  __shared__ double sl[CB * NO];
  float *sW2 = nsm, *sh1 = nsm + NH * S2, *sh2 = sh1 + CB * S2, *sd2 = sh2 + CB * S2, *sd1 = sd2 + CB * S2;
  const int tid = threadIdx.x, b0 = blockIdx.x * CB;
  for (int e = tid; e < CB * NF; e += NH) {
    const int b = e / NF, i = e % NF;
    sx[b][i] = (b0 + b < nb) ? X[(size_t)(n0 + b0 + b) * NF + i] : 0.f;
  }
  __syncthreads();
  net_hidden(P, sx, sW2, sh1, sh2);
  if (tid < CB * NO) {
    const int b = tid / NO, o = tid % NO;
    const bool valid = b0 + b < nb;
    const float y = net_out(P, sh2, b, o);
    const float d = valid ? y - T[(size_t)(n0 + b0 + b) * NO + o] : 0.f;
    sr[b][o] = d * inv_n;
    sl[tid] = 0.5 * (double)d * (double)d * (double)inv_n;
  }
  __syncthreads();
  const int j = tid;
  const float w30 = P[P_W3 + j], w31 = P[P_W3 + NH + j];
  for (int b = 0; b < CB; ++b) {
    const float h = sh2[b * S2 + j];
    sd2[b * S2 + j] = (sr[b][0] * w30 + sr[b][1] * w31) * (1.f - h * h);
  }
  __syncthreads();
  for (int b = 0; b < CB; ++b) {
    float z = 0.f;
    const float *d2 = sd2 + b * S2;
    for (int q = 0; q < NH; ++q) z = fmaf(d2[q], sW2[q * S2 + j], z);
    const float h = sh1[b * S2 + j];
    sd1[b * S2 + j] = z * (1.f - h * h);
  }
  __syncthreads();
  float *out = part + (size_t)blockIdx.x * NP;
  // W2 [q][j]: sum_b d2[b][q] h1[b][j]; thread j writes column j of every row
  for (int q = 0; q < NH; ++q) {
    float z = 0.f;
    for (int b = 0; b < CB; ++b) z = fmaf(sd2[b * S2 + q], sh1[b * S2 + j], z);
    out[P_W2 + q * NH + j] = z;
  }
  float gb2 = 0.f, gb1 = 0.f, g3[NO] = {0.f, 0.f}, g1[NF];
#pragma unroll
  for (int i = 0; i < NF; ++i) g1[i] = 0.f;
  for (int b = 0; b < CB; ++b) {
    gb2 += sd2[b * S2 + j];
    const float d1 = sd1[b * S2 + j];
    gb1 += d1;
#pragma unroll
    for (int i = 0; i < NF; ++i) g1[i] = fmaf(d1, sx[b][i], g1[i]);
    const float h2 = sh2[b * S2 + j];
    g3[0] = fmaf(sr[b][0], h2, g3[0]);
    g3[1] = fmaf(sr[b][1], h2, g3[1]);
  }
  out[P_B2 + j] = gb2;
  out[P_B1 + j] = gb1;
#pragma unroll
  for (int i = 0; i < NF; ++i) out[P_W1 + j * NF + i] = g1[i];
  out[P_W3 + j] = g3[0];
  out[P_W3 + NH + j] = g3[1];
  if (tid < NO) {
    float z = 0.f;
    for (int b = 0; b < CB; ++b) z += sr[b][tid];
    out[P_B3 + tid] = z;
  }
  if (tid == 0) {
    double l = 0.0;
    for (int i = 0; i < CB * NO; ++i) l += sl[i];
    lpart[blockIdx.x] = l;
  }
}

// grad[p] = sum over workgroups of part[wg][p] (fixed order); loss += scale * sum lpart.
__global__ void k_cv_reduce(const float *__restrict__ part, int nwg, float *__restrict__ grad,
                            const double *__restrict__ lpart, double scale, double *__restrict__ loss) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < NP) {
    double s = 0.0;
    for (int g = 0; g < nwg; ++g) s += (double)part[(size_t)g * NP + p];
    grad[p] = (float)s;
  }
  if (p == 0 && loss) {
    double l = 0.0;
    for (int g = 0; g < nwg; ++g) l += lpart[g];
    loss[0] += scale * l;
  }
}

__global__ void k_cv_adam(float *__restrict__ P, const float *__restrict__ grad, float *__restrict__ m,
                          float *__restrict__ v, float lr, float c1, float c2) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= NP) return;
  const float g = grad[p];
  const float mm = 0.9f * m[p] + 0.1f * g;
  const float vv = 0.999f * v[p] + 0.001f * g * g;
  m[p] = mm;
  v[p] = vv;
  P[p] -= lr * (mm / c1) / (sqrtf(vv / c2) + 1e-8f);
}

// Means and (population) deviations of the 8 features and of Re/Im EK over n
// samples; a deviation below 1e-12 is replaced by 1.  One workgroup.
__global__ __launch_bounds__(kThreads) void k_cv_stats(const double *__restrict__ feat,
                                                       const double2 *__restrict__ ek, long n,
                                                       double *__restrict__ norm) {
  __shared__ double red[4 * (NF + NO)];
  __shared__ double mean[NF + NO];
  double acc[NF + NO];
#pragma unroll
  for (int c = 0; c < NF + NO; ++c) acc[c] = 0.0;
  for (long s = threadIdx.x; s < n; s += blockDim.x) {
#pragma unroll
    for (int c = 0; c < NF; ++c) acc[c] += feat[s * NF + c];
    acc[NF] += ek[s].x;
    acc[NF + 1] += ek[s].y;
  }
  block_sum<NF + NO>(acc, red);
  if (threadIdx.x == 0)
    for (int c = 0; c < NF + NO; ++c) mean[c] = acc[c] / (double)n;
  __syncthreads();
#pragma unroll
  for (int c = 0; c < NF + NO; ++c) acc[c] = 0.0;
  for (long s = threadIdx.x; s < n; s += blockDim.x) {
#pragma unroll
    for (int c = 0; c < NF; ++c) {
      const double d = feat[s * NF + c] - mean[c];
      acc[c] += d * d;
    }
    const double dr = ek[s].x - mean[NF], di = ek[s].y - mean[NF + 1];
    acc[NF] += dr * dr;
    acc[NF + 1] += di * di;
  }
  block_sum<NF + NO>(acc, red);
  if (threadIdx.x == 0) {
    for (int c = 0; c < NF + NO; ++c) {
      double sd = sqrt(acc[c] / (double)n);
      if (!(sd >= 1e-12)) sd = 1.0;
      const int mo = c < NF ? c : 2 * NF + (c - NF);
      const int so = c < NF ? NF + c : 2 * NF + NO + (c - NF);
      norm[mo] = mean[c];
      norm[so] = sd;
    }
  }
}

__global__ void k_cv_standardise(const double *__restrict__ feat, const double2 *__restrict__ ek, long n,
                                 const double *__restrict__ norm, float *__restrict__ X, float *__restrict__ T) {
  const long s = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (s >= n) return;
#pragma unroll
  for (int c = 0; c < NF; ++c) X[s * NF + c] = (float)((feat[s * NF + c] - norm[c]) / norm[NF + c]);
  T[s * NO + 0] = (float)((ek[s].x - norm[2 * NF]) / norm[2 * NF + NO]);
  T[s * NO + 1] = (float)((ek[s].y - norm[2 * NF + 1]) / norm[2 * NF + NO + 1]);
}

// Initial parameters: Glorot-uniform weights (limit sqrt(6 / (fan_in + fan_out)))
// from a SplitMix64 hash of (seed, index), zero biases; normalisation = identity.
__global__ void k_cv_init(float *__restrict__ P, double *__restrict__ norm, unsigned long long seed) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < kCvNorm) norm[p] = (p >= NF && p < 2 * NF) || p >= 2 * NF + NO ? 1.0 : 0.0;
  if (p >= NP) return;
  int fin = 0, fout = 0;
  if (p < P_B1) { fin = NF; fout = NH; }
  else if (p >= P_W2 && p < P_B2) { fin = NH; fout = NH; }
  else if (p >= P_W3 && p < P_B3) { fin = NH; fout = NO; }
  if (fin == 0) {
    P[p] = 0.f;
    return;
  }
  const double u = (double)(splitmix64(seed + (unsigned long long)p * kGolden) >> 11) * 0x1p-53;  // [0, 1)
  const double lim = sqrt(6.0 / (double)(fin + fout));
  P[p] = (float)((2.0 * u - 1.0) * lim);
}

__global__ void k_cv_zero(unsigned int *__restrict__ p, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) p[e] = 0u;
}

// ---- launchers ------------------------------------------------------------------
hipError_t launch_cv_init(const System &s, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_cv_init, dim3((NP + 255) / 256), dim3(256), 0, st, s.cv_params, s.cv_norm,
                     (unsigned long long)seed);
  return hipGetLastError();
}

hipError_t launch_cv_zero(void *p, size_t bytes, hipStream_t st) {
  const long n = (long)(bytes / 4);
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cv_zero, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, static_cast<unsigned int *>(p), n);
  return hipGetLastError();
}

hipError_t cv_enable_lds() {
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(k_cv_predict),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)(NH * S2 + 2 * CB * S2) * 4);
  if (e != hipSuccess) return e;
  return hipFuncSetAttribute(reinterpret_cast<const void *>(k_cv_grad), hipFuncAttributeMaxDynamicSharedMemorySize,
                             (int)kNetLds);
}

hipError_t launch_cv_features(const System &s, int W, double *feat, hipStream_t st) {
  // sum_s Tr(K_s Theta_s), a trace of the same form as the one-body energy
  hipError_t e = launch_trace_half(s.KtT, s.theta, W, (long)s.M * s.Nt, s.cv_lin, st);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cv_features, dim3(W), dim3(kThreads), 0, st, s.fbpart, s.fb_slices, s.G, W, s.lmf, s.e1,
                     s.ej, s.logo_new, s.cv_lin, feat);
  return hipGetLastError();
}

hipError_t launch_cv_predict(const System &s, const double *feat, long n, double2 *f, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cv_predict, dim3((unsigned)((n + CB - 1) / CB)), dim3(NH), (NH * S2 + 2 * CB * S2) * 4, st,
                     s.cv_params, s.cv_norm, feat, (int)n, f);
  return hipGetLastError();
}

hipError_t launch_cv_subset(const System &s, int W, int k, uint64_t seed, hipStream_t st) {
  hipLaunchKernelGGL(k_cv_subset, dim3(1), dim3(1024), 0, st, W, k, (unsigned long long)seed,
                     reinterpret_cast<unsigned long long *>(s.cv_counter),
                     reinterpret_cast<unsigned long long *>(s.cv_counter) + 1, s.cv_sel, s.cv_pos);
  return hipGetLastError();
}

hipError_t launch_cv_gather(const System &s, int k, hipStream_t st) {
  const long per = (long)s.M * s.Nt, n = (long)k * per;
  if (n == 0) return hipSuccess;
  hipLaunchKernelGGL(k_cv_gather, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.theta, s.cv_sel, k, per,
                     s.cv_theta);
  return hipGetLastError();
}

hipError_t launch_cv_combine(const System &s, int W, int k, double2 *e_out, hipStream_t st) {
  hipLaunchKernelGGL(k_cv_combine, dim3(W), dim3(kThreads), 0, st, s.e1, s.ej, s.ekpart, s.ex_stride,
                     s.ex_nparts[0], s.ex_nparts[1], s.cv_f, s.cv_pos, (double)W / (double)k, s.stat_new, e_out);
  return hipGetLastError();
}

hipError_t launch_cv_ek(const System &s, int W, double2 *ek, hipStream_t st) {
  hipLaunchKernelGGL(k_cv_ek, dim3(W), dim3(kThreads), 0, st, s.ekpart, s.ex_stride, s.ex_nparts[0], s.ex_nparts[1],
                     ek);
  return hipGetLastError();
}

hipError_t launch_cv_stats(const double *feat, const double2 *ek, long n, double *norm, hipStream_t st) {
  hipLaunchKernelGGL(k_cv_stats, dim3(1), dim3(kThreads), 0, st, feat, ek, n, norm);
  return hipGetLastError();
}

hipError_t launch_cv_standardise(const double *feat, const double2 *ek, long n, const double *norm, float *X,
                                 float *T, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_cv_standardise, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, feat, ek, n, norm, X, T);
  return hipGetLastError();
}

int cv_grad_workgroups(long nb) { return (int)((nb + CB - 1) / CB); }

hipError_t launch_cv_grad(const float *P, const float *X, const float *T, long n0, long nb, float *part,
                          double *lpart, float *grad, double loss_scale, double *loss, hipStream_t st) {
  const int nwg = cv_grad_workgroups(nb);
  hipLaunchKernelGGL(k_cv_grad, dim3(nwg), dim3(NH), kNetLds, st, P, X, T, (int)n0, (int)nb, 1.0f / (float)nb, part,
                     lpart);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_cv_reduce, dim3((NP + 255) / 256), dim3(256), 0, st, part, nwg, grad, lpart, loss_scale, loss);
  return hipGetLastError();
}

hipError_t launch_cv_adam(float *P, const float *grad, float *m, float *v, double lr, long t, hipStream_t st) {
  const double c1 = 1.0 - std::pow(0.9, (double)t), c2 = 1.0 - std::pow(0.999, (double)t);
  hipLaunchKernelGGL(k_cv_adam, dim3((NP + 255) / 256), dim3(256), 0, st, P, grad, m, v, (float)lr, (float)c1,
                     (float)c2);
  return hipGetLastError();
}

}  // namespace afqmc
