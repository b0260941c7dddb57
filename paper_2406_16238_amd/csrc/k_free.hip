// Free projection (the fp-AFQMC section): the per-walker kernels that differ
// from the phaseless step.  The propagation itself (V_HS, B1, Taylor series,
// overlap) is the phaseless step's, fed with the bare fields.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

// ---- fields: y = x (no force bias) -------------------------------------------
// Rows of the V_HS product as in the phaseless epilogue, for a real y:
// yp[w][0][g] = sqrt(dt) Im y_g = 0, yp[w][1][g] = -sqrt(dt) x_g.  Also
// wsc[w][4] = sum_g x_g l_g (the mean-field phase); the other five sums are 0.
// A walker whose x has a NaN/Inf is flagged and propagated with x = 0.
__global__ __launch_bounds__(kThreads) void k_free_fields(const double *__restrict__ lmf,
                                                         const double *__restrict__ x, int G, double sqdt,
                                                         double *__restrict__ yp, double *__restrict__ wsc,
                                                         uint32_t *__restrict__ flags) {
  __shared__ double red[4 * 1];
  __shared__ int sbad;
  const int w = blockIdx.x, tid = threadIdx.x;
  const double *xw = x + (size_t)w * G;
  double bad[1] = {0.0};
  for (int g = tid; g < G; g += blockDim.x)
    if (!isfinite(xw[g])) bad[0] = 1.0;
  block_sum<1>(bad, red);
  if (tid == 0) sbad = bad[0] > 0.0;
  __syncthreads();
  const bool nonfinite = sbad;
  double acc[1] = {0.0};
  for (int g = tid; g < G; g += blockDim.x) {
    const double xv = nonfinite ? 0.0 : xw[g];
    yp[((size_t)w * 2 + 0) * G + g] = 0.0;
    yp[((size_t)w * 2 + 1) * G + g] = -sqdt * xv;
    acc[0] += xv * lmf[g];
  }
  block_sum<1>(acc, red);
  if (tid == 0) {
    double *o = wsc + (size_t)w * 6;
    o[0] = o[1] = o[2] = o[3] = o[5] = 0.0;
    o[4] = acc[0];
    if (nonfinite) flags[w] |= AFQMC_W_NONFINITE;
  }
}

hipError_t launch_free_fields(const System &s, const double *x, int W, uint32_t *flags, hipStream_t st) {
  hipLaunchKernelGGL(k_free_fields, dim3(W), dim3(kThreads), 0, st, s.lmf, x, s.G, s.sqdt, s.yp, s.wsc, flags);
  return hipGetLastError();
}

// ---- amplitude: a <- a + log S - dt (C - E_T) ---------------------------------
// log S = log<Psi_T|phi'> - log<Psi_T|phi> + i sqrt(dt) x.l (eq. ovlp_ratio
// with y = x).  Im a is reduced to [-pi, pi] so that it keeps its precision
// over long runs.  A singular new overlap flags the walker and leaves a and
// log_ovlp as they were.
__global__ void k_free_amplitude(double2 *__restrict__ logo, const double2 *__restrict__ logo_new,
                                 const uint32_t *__restrict__ stat_new, const double *__restrict__ wsc, double sqdt,
                                 double dt, double const_c, const double *__restrict__ eshift, int W,
                                 double2 *__restrict__ amp, uint32_t *__restrict__ flags) {
  const int w = blockIdx.x * blockDim.x + threadIdx.x;
  if (w >= W) return;
  const double dshift = -dt * (const_c - eshift[0]);
  if (stat_new[w]) {
    flags[w] |= stat_new[w];
    return;
  }
  const double2 a = amp[w], o = logo[w], n = logo_new[w];
  const double re = a.x + (n.x - o.x) + dshift;
  double im = a.y + (n.y - o.y) + sqdt * wsc[(size_t)w * 6 + 4];
  const double two_pi = 6.283185307179586476925286766559;
  im -= two_pi * rint(im / two_pi);
  amp[w] = make_double2(re, im);
  logo[w] = n;
}

hipError_t launch_free_amplitude(const System &s, const afqmc_walkers &wk, double2 *amp, int W, hipStream_t st) {
  hipLaunchKernelGGL(k_free_amplitude, dim3((W + 255) / 256), dim3(256), 0, st,
                     reinterpret_cast<double2 *>(wk.log_ovlp), s.logo_new, s.stat_new, s.wsc, s.sqdt, s.dt,
                     s.const_c, s.eshift, W, amp, wk.flags);
  return hipGetLastError();
}

// ---- estimator ------------------------------------------------------------------
// One workgroup: r = max Re a over the walkers that count, then the complex
// sums of z = weight e^{a - r} times (E, 1, E1, E2), each thread over a fixed
// stride of walkers and a fixed reduction tree.
__global__ __launch_bounds__(kThreads) void k_free_estimator(const double *__restrict__ weight,
                                                            const uint32_t *__restrict__ flags,
                                                            const double2 *__restrict__ amp,
                                                            const double2 *__restrict__ e, int W,
                                                            double *__restrict__ est) {
  __shared__ double red[4 * 9];
  __shared__ double wmax[kThreads / 64];
  const int tid = threadIdx.x, lane = tid & 63, wid = tid >> 6;
  auto counts = [&](int w) {
    const double2 a = amp[w];
    return weight[w] > 0.0 && !(flags[w] & (AFQMC_W_SINGULAR | AFQMC_W_NONFINITE)) && isfinite(a.x) &&
           isfinite(a.y);
  };
  double m = -INFINITY;
  for (int w = tid; w < W; w += blockDim.x)
    if (counts(w)) m = fmax(m, amp[w].x);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) m = fmax(m, __shfl_down(m, o, 64));
  if (lane == 0) wmax[wid] = m;
  __syncthreads();
  double r = wmax[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) r = fmax(r, wmax[k]);
  if (!(r > -INFINITY)) r = 0.0;

  double acc[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
  for (int w = tid; w < W; w += blockDim.x) {
    if (!counts(w)) continue;
    const double2 a = amp[w];
    const double mag = weight[w] * exp(a.x - r);
    double sn, cs;
    sincos(a.y, &sn, &cs);
    const double zr = mag * cs, zi = mag * sn;
    const double2 E = e[(size_t)w * 3 + 0], E1 = e[(size_t)w * 3 + 1], E2 = e[(size_t)w * 3 + 2];
    acc[0] += zr * E.x - zi * E.y;
    acc[1] += zr * E.y + zi * E.x;
    acc[2] += zr;
    acc[3] += zi;
    acc[4] += zr * E1.x - zi * E1.y;
    acc[5] += zr * E1.y + zi * E1.x;
    acc[6] += zr * E2.x - zi * E2.y;
    acc[7] += zr * E2.y + zi * E2.x;
    acc[8] += 1.0;
  }
  block_sum<9>(acc, red);
  if (tid == 0) {
    for (int i = 0; i < 8; ++i) est[i] = acc[i];
    est[8] = r;
    est[9] = acc[8];
  }
}

hipError_t launch_free_estimator(const double *weight, const uint32_t *flags, const double2 *amp, const double2 *e,
                                 int W, double *est, hipStream_t st) {
  hipLaunchKernelGGL(k_free_estimator, dim3(1), dim3(kThreads), 0, st, weight, flags, amp, e, W, est);
  return hipGetLastError();
}

}  // namespace afqmc
