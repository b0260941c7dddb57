// Population control by a comb (the population-control step of the
// simulation loop of Sec. 3.1; the paper does not fix the method): with cumulative weights C_i
// summed in walker order and total Wt, W teeth at (u + k) Wt / W for one
// uniform u in [0, 1); tooth k selects the first walker i with C_i > tooth, new
// walker k is a copy of it (orbitals, log-overlap, flags) and every weight
// becomes Wt / W.  The prefix sum runs in one thread, in walker order, so the
// choice is reproducible and equals a sequential host computation bit for bit.
#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

// One workgroup.  cum [W] scratch; parents [W] out; weight rewritten.
__global__ __launch_bounds__(kThreads) void k_comb(double *__restrict__ weight, int W, const double *__restrict__ u,
                                                   double *__restrict__ cum, int *__restrict__ parents) {
  __shared__ double total_s;
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int i = 0; i < W; ++i) {
      c += weight[i];
      cum[i] = c;
    }
    total_s = c;
  }
  __syncthreads();
  const double total = total_s;
  const double off = u[0];
  const bool live = total > 0.0;
  const double step = total / W;
  for (int k = threadIdx.x; k < W; k += blockDim.x) {
    int p = k;
    if (live) {
      const double tooth = (off + k) * step;
      int lo = 0, hi = W - 1;  // first i with cum[i] > tooth, at most W - 1
      while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (cum[mid] > tooth) hi = mid;
        else lo = mid + 1;
      }
      p = lo;
    }
    parents[k] = p;
  }
  __syncthreads();
  if (live)
    for (int k = threadIdx.x; k < W; k += blockDim.x) weight[k] = step;
}

// out[k] = in[parents[k]] for whole walkers of `per` double2 (and the scalars)
__global__ void k_gather_walkers(const double2 *__restrict__ phi, const double2 *__restrict__ logo,
                                 const uint32_t *__restrict__ flags, const int *__restrict__ parents, int W, long per,
                                 double2 *__restrict__ phi_out, double2 *__restrict__ logo_out,
                                 uint32_t *__restrict__ flags_out) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)W * per) return;
  const long k = e / per, r = e - k * per;
  const long src = parents[k];
  phi_out[e] = phi[src * per + r];
  if (r == 0) {
    logo_out[k] = logo[src];
    flags_out[k] = flags[src];
  }
}

__global__ void k_scatter_back(const double2 *__restrict__ phi_in, const double2 *__restrict__ logo_in,
                               const uint32_t *__restrict__ flags_in, int W, long per, double2 *__restrict__ phi,
                               double2 *__restrict__ logo, uint32_t *__restrict__ flags) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= (long)W * per) return;
  phi[e] = phi_in[e];
  if (e % per == 0) {
    const long k = e / per;
    logo[k] = logo_in[k];
    flags[k] = flags_in[k];
  }
}

hipError_t launch_comb(const System &s, double *weight, double2 *phi, double2 *logo, uint32_t *flags, const double *u,
                       int *parents_out, hipStream_t st) {
  const int W = s.W;
  const long per = (long)s.M * s.Nt, n = (long)W * per;
  int *parents = parents_out ? parents_out : s.cv_pos;
  hipLaunchKernelGGL(k_comb, dim3(1), dim3(kThreads), 0, st, weight, W, u, s.wsc, parents);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  hipLaunchKernelGGL(k_gather_walkers, dim3(blocks), dim3(256), 0, st, phi, logo, flags, parents, W, per, s.tA,
                     s.logo_now, s.stat_now);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(k_scatter_back, dim3(blocks), dim3(256), 0, st, s.tA, s.logo_now, s.stat_now, W, per, phi, logo,
                     flags);
  return hipGetLastError();
}

}  // namespace afqmc
