// Per-walker epilogues of the phaseless step and of the local energy, the
// deterministic estimator reduction, and small set-up kernels.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

// ---- force-bias epilogue of the propagation (Sec. 2, eqs. fb and Bprop) -----
// vbias_g = sum over split-K slices; xbar_g = i sqrt(dt) (vbias_g - l_g), capped
// in modulus at fb_cap; y = x - xbar.  Writes the rows of the V_HS product,
// yp[w][0][g] = sqrt(dt) Im y_g, yp[w][1][g] = -sqrt(dt) Re y_g, so that
// sum_g yp[w][c][g] L^g are the real (c = 0) and imaginary (c = 1) planes of
// sqrt(dt) V_HS = -i sqrt(dt) sum_g y_g L^g.  Also reduces, per walker,
// sum_g x_g xbar_g, sum_g xbar_g^2 and sum_g y_g l_g.  A walker whose x has a
// NaN/Inf is flagged and propagated with x = 0.
__global__ __launch_bounds__(kThreads) void k_fb_propagate(const double2 *__restrict__ part, int ksplit,
                                                          const double *__restrict__ lmf,
                                                          const double *__restrict__ x, int G, int W,
                                                          double sqdt, double cap, double *__restrict__ yp,
                                                          double *__restrict__ wsc,
                                                          uint32_t *__restrict__ flags) {
  __shared__ double red[4 * 6];
  const int w = blockIdx.x, tid = threadIdx.x;
  const double *xw = x + (size_t)w * G;
  double bad[1] = {0.0};
  for (int g = tid; g < G; g += blockDim.x)
    if (!isfinite(xw[g])) bad[0] = 1.0;
  block_sum<1>(bad, red);
  __shared__ int sbad;
  if (tid == 0) sbad = bad[0] > 0.0;
  __syncthreads();
  const bool nonfinite = sbad;

  double acc[6] = {0, 0, 0, 0, 0, 0};
  for (int g = tid; g < G; g += blockDim.x) {
    double2 vb = make_double2(0.0, 0.0);
    for (int s = 0; s < ksplit; ++s) vb = cadd(vb, part[((size_t)s * W + w) * G + g]);
    const double l = lmf[g];
    double2 xb = make_double2(-sqdt * vb.y, sqdt * (vb.x - l));
    if (cap > 0.0) {
      const double m = sqrt(cabs2(xb));
      if (m > cap) xb = cscale(xb, cap / m);
    }
    const double xv = nonfinite ? 0.0 : xw[g];
    const double2 y = make_double2(xv - xb.x, -xb.y);
    yp[((size_t)w * 2 + 0) * G + g] = sqdt * y.y;
    yp[((size_t)w * 2 + 1) * G + g] = -sqdt * y.x;
    acc[0] += xv * xb.x;
    acc[1] += xv * xb.y;
    acc[2] += xb.x * xb.x - xb.y * xb.y;
    acc[3] += 2.0 * xb.x * xb.y;
    acc[4] += y.x * l;
    acc[5] += y.y * l;
  }
  block_sum<6>(acc, red);
  if (tid == 0) {
    for (int i = 0; i < 6; ++i) wsc[(size_t)w * 6 + i] = acc[i];
    if (nonfinite) flags[w] |= AFQMC_W_NONFINITE;
  }
}

hipError_t launch_fb_propagate_epilogue(const System &s, const Options &o, const double *x, int W,
                                        uint32_t *flags, int nslices, hipStream_t st) {
  hipLaunchKernelGGL(k_fb_propagate, dim3(W), dim3(kThreads), 0, st, s.fbpart, nslices, s.lmf, x, s.G,
                     W, s.sqdt, o.fb_cap, s.yp, s.wsc, flags);
  return hipGetLastError();
}

// ---- force-bias epilogue of the local energy: EJ = 1/2 sum_g vbias_g^2 --------
__global__ __launch_bounds__(kThreads) void k_fb_energy(const double2 *__restrict__ part, int ksplit, int G,
                                                       int W, double2 *__restrict__ ej,
                                                       double2 *__restrict__ vbias_out) {
  __shared__ double red[4 * 2];
  const int w = blockIdx.x, tid = threadIdx.x;
  double acc[2] = {0.0, 0.0};
  for (int g = tid; g < G; g += blockDim.x) {
    double2 vb = make_double2(0.0, 0.0);
    for (int s = 0; s < ksplit; ++s) vb = cadd(vb, part[((size_t)s * W + w) * G + g]);
    if (vbias_out) vbias_out[(size_t)w * G + g] = vb;
    acc[0] += vb.x * vb.x - vb.y * vb.y;
    acc[1] += 2.0 * vb.x * vb.y;
  }
  block_sum<2>(acc, red);
  if (tid == 0) ej[w] = make_double2(0.5 * acc[0], 0.5 * acc[1]);
}

hipError_t launch_fb_energy_epilogue(const System &s, int W, double2 *vbias_out, int nslices, hipStream_t st) {
  hipLaunchKernelGGL(k_fb_energy, dim3(W), dim3(kThreads), 0, st, s.fbpart, nslices, s.G, W, s.ej,
                     vbias_out);
  return hipGetLastError();
}

// ---- weight update (Sec. 2, eq. weight_update, the phaseless and hybrid
// importance functions, eq. ovlp_ratio) --------------------------------------
// log S = log<Psi_T|phi'> - log<Psi_T|phi> + i sqrt(dt) sum_g y_g l_g,
// theta = Im log S, |I| = exp(Re log S + Re(sum x.xbar - sum xbar^2 / 2)),
// w <- w |I| max(0, cos theta) exp(-dt (C - E_T)).
// E_T is read from device memory (eshift[0]) so that it can follow the running
// estimate without the host and without invalidating recorded graphs.
__global__ void k_weight_update(const double2 *__restrict__ logo_now, const double2 *__restrict__ logo_new,
                                const uint32_t *__restrict__ stat_now, const uint32_t *__restrict__ stat_new,
                                const double *__restrict__ wsc, double sqdt, double dt, double const_c,
                                const double *__restrict__ eshift, int W, double *__restrict__ weight,
                                double2 *__restrict__ logo, uint32_t *__restrict__ flags) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double shift_factor = exp(-dt * (const_c - eshift[0]));
  uint32_t f = flags[w];
  const uint32_t sing = stat_now[w] | stat_new[w];
  if (sing) {
    weight[w] = 0.0;
    flags[w] = f | sing;
    return;
  }
  const double *sc = wsc + (size_t)w * 6;
  const double2 a = logo_now[w], b = logo_new[w];
  const double ls_re = (b.x - a.x) - sqdt * sc[5];
  const double ls_im = (b.y - a.y) + sqdt * sc[4];
  const double lnI = ls_re + sc[0] - 0.5 * sc[2];
  const double c = cos(ls_im);
  double nw = weight[w] * exp(lnI) * (c > 0.0 ? c : 0.0) * shift_factor;
  if (!(c > 0.0)) {
    f |= AFQMC_W_DEAD;
    nw = 0.0;
  }
  if (f & AFQMC_W_NONFINITE) nw = 0.0;
  weight[w] = nw;
  logo[w] = b;
  flags[w] = f;
}

hipError_t launch_weight_update(const System &s, const afqmc_walkers &wk, int W, hipStream_t st) {
  hipLaunchKernelGGL(k_weight_update, dim3((W + 255) / 256), dim3(256), 0, st, s.logo_now, s.logo_new,
                     s.stat_now, s.stat_new, s.wsc, s.sqdt, s.dt, s.const_c, s.eshift, W, wk.weight,
                     reinterpret_cast<double2 *>(wk.log_ovlp), wk.flags);
  return hipGetLastError();
}

// ---- one-body energy: E1 = ecore + sum_{q,i'} htT[q][i'] Theta[w][q][i'] ------
// One workgroup of sixteen waves per walker: with one workgroup per CU, four
// waves left the loads of a walker's Theta too few in flight.
constexpr int kE1Threads = 1024;
__global__ __launch_bounds__(kE1Threads) void k_energy_e1(const double *__restrict__ htT,
                                                         const double2 *__restrict__ theta, long K,
                                                         double ecore, double2 *__restrict__ e1) {
  __shared__ double red[kE1Threads / 64 * 2];
  const int w = blockIdx.x;
  const double2 *th = theta + (size_t)w * K;
  double acc[2] = {0.0, 0.0};
  for (long k = threadIdx.x; k < K; k += blockDim.x) {
    const double h = htT[k];
    const double2 t = th[k];
    acc[0] = fma(h, t.x, acc[0]);
    acc[1] = fma(h, t.y, acc[1]);
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) e1[w] = make_double2(ecore + acc[0], acc[1]);
}

hipError_t launch_energy_e1(const System &s, const double2 *theta, int W, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_e1, dim3(W), dim3(kE1Threads), 0, st, s.htT, theta, (long)s.M * s.Nt, s.ecore,
                     s.e1);
  return hipGetLastError();
}

hipError_t launch_trace_half(const double *mat, const double2 *theta, int W, long K, double2 *out, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_e1, dim3(W), dim3(kE1Threads), 0, st, mat, theta, K, 0.0, out);
  return hipGetLastError();
}

// ---- combine: E2 = EJ + sum of exchange partials (fixed order), E = E1 + E2 ---
__global__ __launch_bounds__(kThreads) void k_energy_combine(const double2 *__restrict__ e1,
                                                            const double2 *__restrict__ ej,
                                                            const double2 *__restrict__ ekpart, int stride,
                                                            int n0, int n1, const uint32_t *__restrict__ stat,
                                                            double2 *__restrict__ e_out) {
  __shared__ double red[4 * 2];
  const int w = blockIdx.x;
  const double2 *p = ekpart + (size_t)w * 2 * stride;
  double acc[2] = {0.0, 0.0};
  for (int k = threadIdx.x; k < n0; k += blockDim.x) {
    acc[0] += p[k].x;
    acc[1] += p[k].y;
  }
  for (int k = threadIdx.x; k < n1; k += blockDim.x) {
    acc[0] += p[stride + k].x;
    acc[1] += p[stride + k].y;
  }
  block_sum<2>(acc, red);
  if (threadIdx.x == 0) {
    const double2 a = e1[w], j = ej[w];
    const double2 e2 = make_double2(j.x + acc[0], j.y + acc[1]);
    const bool sing = stat[w] != 0u;  // <Psi_T|phi> = 0: no local energy, report zeros
    const double2 z = make_double2(0.0, 0.0);
    e_out[(size_t)w * 3 + 0] = sing ? z : cadd(a, e2);
    e_out[(size_t)w * 3 + 1] = sing ? z : a;
    e_out[(size_t)w * 3 + 2] = sing ? z : e2;
  }
}

hipError_t launch_energy_combine(const System &s, int W, double2 *e_out, hipStream_t st) {
  hipLaunchKernelGGL(k_energy_combine, dim3(W), dim3(kThreads), 0, st, s.e1, s.ej, s.ekpart, s.ex_stride,
                     s.ex_nparts[0], s.ex_nparts[1], s.stat_new, e_out);
  return hipGetLastError();
}

// ---- estimator record: ENumer, EDenom, E1Body, E2Body over walkers with w > 0 --
__global__ __launch_bounds__(kThreads) void k_estimator(const double *__restrict__ weight,
                                                       const double2 *__restrict__ e, int W,
                                                       double *__restrict__ est) {
  __shared__ double red[4 * 4];
  double acc[4] = {0, 0, 0, 0};
  for (int w = threadIdx.x; w < W; w += blockDim.x) {
    const double wt = weight[w];
    if (wt > 0.0) {
      acc[0] += wt * e[(size_t)w * 3 + 0].x;
      acc[1] += wt;
      acc[2] += wt * e[(size_t)w * 3 + 1].x;
      acc[3] += wt * e[(size_t)w * 3 + 2].x;
    }
  }
  block_sum<4>(acc, red);
  if (threadIdx.x == 0)
    for (int i = 0; i < 4; ++i) est[i] = acc[i];
}

hipError_t launch_estimator(const double *weight, const double2 *e_out, int W, double *est, hipStream_t st) {
  hipLaunchKernelGGL(k_estimator, dim3(1), dim3(kThreads), 0, st, weight, e_out, W, est);
  return hipGetLastError();
}

// ---- energy shift ------------------------------------------------------------
__global__ void k_set_scalar(double *__restrict__ p, double v) {
  if (threadIdx.x == 0 && blockIdx.x == 0) p[0] = v;
}

hipError_t launch_set_e_shift(const System &s, double e_shift, hipStream_t st) {
  hipLaunchKernelGGL(k_set_scalar, dim3(1), dim3(64), 0, st, s.eshift, e_shift);
  return hipGetLastError();
}

// Feedback of a block (the simulation loop of Sec. 3.1): E_T <- sum_k ENumer_k /
// sum_k EDenom_k over the block's estimator records est[k][4], summed in step
// order by one thread; kept when the denominator is not positive or the ratio
// is not finite.
__global__ void k_block_e_shift(const double *__restrict__ est, int nsteps, double *__restrict__ eshift) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double num = 0.0, den = 0.0;
  for (int k = 0; k < nsteps; ++k) {
    num += est[(size_t)k * 4 + 0];
    den += est[(size_t)k * 4 + 1];
  }
  if (den > 0.0) {
    const double e = num / den;
    if (isfinite(e)) eshift[0] = e;
  }
}

hipError_t launch_block_e_shift(const System &s, const double *est, int nsteps, hipStream_t st) {
  hipLaunchKernelGGL(k_block_e_shift, dim3(1), dim3(64), 0, st, est, nsteps, s.eshift);
  return hipGetLastError();
}

// ---- set-up helpers -----------------------------------------------------------
__global__ __launch_bounds__(kThreads) void k_row_dot(const double *__restrict__ A,
                                                     const double *__restrict__ v, long len,
                                                     double *__restrict__ out) {
  __shared__ double red[4];
  const double *a = A + (size_t)blockIdx.x * len;
  double acc[1] = {0.0};
  for (long k = threadIdx.x; k < len; k += blockDim.x) acc[0] = fma(a[k], v[k], acc[0]);
  block_sum<1>(acc, red);
  if (threadIdx.x == 0) out[blockIdx.x] = acc[0];
}

hipError_t launch_row_dot(const double *A, const double *v, long len, int rows, double *out, hipStream_t st) {
  hipLaunchKernelGGL(k_row_dot, dim3(rows), dim3(kThreads), 0, st, A, v, len, out);
  return hipGetLastError();
}

__global__ void k_sum_slices(const double *__restrict__ parts, int nslices, long n, double alpha,
                             double *__restrict__ inout) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int k = 0; k < nslices; ++k) s += parts[(size_t)k * n + i];
  inout[i] += alpha * s;
}

hipError_t launch_sum_slices(const double *parts, int nslices, long n, double alpha, double *inout,
                             hipStream_t st) {
  hipLaunchKernelGGL(k_sum_slices, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, parts, nslices, n,
                     alpha, inout);
  return hipGetLastError();
}

__global__ void k_add_identity(double *A, int M, double diag) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < M) A[(size_t)i * M + i] += diag;
}

hipError_t launch_add_identity(double *A, int M, double diag, hipStream_t st) {
  hipLaunchKernelGGL(k_add_identity, dim3((M + 255) / 256), dim3(256), 0, st, A, M, diag);
  return hipGetLastError();
}

__global__ void k_fill_zero2(double2 *__restrict__ p, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = make_double2(0.0, 0.0);
}

hipError_t launch_zero2(double2 *p, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_zero2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

// Deterministic values in [-1/2, 1/2) from an integer hash of the index, for
// timing kernels on data with realistic bit patterns.
__global__ void k_fill_pattern2(double2 *__restrict__ p, long n) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  unsigned long long z = (unsigned long long)e * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
  z = (z ^ (z >> 31)) * 0xD6E8FEB86659FD93ull;
  z ^= z >> 32;
  const double a = (double)(z & 0xFFFFFFFFull) * 0x1p-32 - 0.5, b = (double)(z >> 32) * 0x1p-32 - 0.5;
  p[e] = make_double2(a, b);
}

hipError_t launch_fill_pattern2(double2 *p, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_fill_pattern2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, p, n);
  return hipGetLastError();
}

__global__ void k_axpby(const double *__restrict__ x, double a, double *__restrict__ y, double b, long n) {
  const long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}

hipError_t launch_axpby(const double *x, double a, double *y, double b, long n, hipStream_t st) {
  hipLaunchKernelGGL(k_axpby, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, x, a, y, b, n);
  return hipGetLastError();
}

}  // namespace afqmc
