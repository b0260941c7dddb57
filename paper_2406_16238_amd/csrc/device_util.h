// Device helpers: complex arithmetic on interleaved double2 and deterministic
// workgroup reductions built from 64-lane wavefront shuffles.
#pragma once

#include <hip/hip_runtime.h>

namespace afqmc {

__device__ __forceinline__ double2 cadd(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 csub(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 cmul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ double2 cscale(double2 a, double s) { return make_double2(a.x * s, a.y * s); }
// a / b by Smith's scaling, safe for |b| over a wide range
__device__ __forceinline__ double2 cdiv(double2 a, double2 b) {
  if (fabs(b.x) >= fabs(b.y)) {
    double r = b.y / b.x, d = b.x + b.y * r;
    return make_double2((a.x + a.y * r) / d, (a.y - a.x * r) / d);
  }
  double r = b.x / b.y, d = b.x * r + b.y;
  return make_double2((a.x * r + a.y) / d, (a.y * r - a.x) / d);
}
__device__ __forceinline__ double cabs2(double2 a) { return a.x * a.x + a.y * a.y; }

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_down(v, o, 64);
  return v;
}

// One DPP step of a wave reduction on a double (both 32-bit halves moved by
// the same control); lanes that the row mask leaves out read 0.
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ double dpp_double(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), CTRL, ROWS, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

// Sum over the 64 lanes, valid in lane 63: quad swaps and the row mirrors
// give every lane its row's sum, the row broadcasts of lanes 15 and 31 add
// the rows up.  A fixed order, and no LDS traffic (unlike a shuffle tree).
__device__ __forceinline__ double wave_sum_dpp(double v) {
  v += dpp_double<0xB1>(v);         // quad_perm [1,0,3,2]
  v += dpp_double<0x4E>(v);         // quad_perm [2,3,0,1]
  v += dpp_double<0x141>(v);        // row_half_mirror
  v += dpp_double<0x140>(v);        // row_mirror
  v += dpp_double<0x142, 0xA>(v);   // row_bcast:15 into rows 1 and 3
  v += dpp_double<0x143, 0xC>(v);   // row_bcast:31 into rows 2 and 3
  return v;
}

// Largest value over the 64 lanes with its index, ties to the smaller index
// (values >= 0; lanes with nothing hold -1), valid in lane 63; the same DPP
// steps as wave_sum_dpp, lanes the row mask leaves out reading (-1, INT_MAX).
template <int CTRL, int ROWS = 0xF>
__device__ __forceinline__ void dpp_argmax_step(double &best, int &bi) {
  const long long b = __double_as_longlong(best), none = __double_as_longlong(-1.0);
  const int lo = __builtin_amdgcn_update_dpp((int)none, (int)b, CTRL, ROWS, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp((int)(none >> 32), (int)(b >> 32), CTRL, ROWS, 0xF, false);
  const double ob = __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
  const int oi = __builtin_amdgcn_update_dpp(0x7fffffff, bi, CTRL, ROWS, 0xF, false);
  if (ob > best || (ob == best && oi < bi)) {
    best = ob;
    bi = oi;
  }
}
__device__ __forceinline__ void wave_argmax_dpp(double &best, int &bi) {
  dpp_argmax_step<0xB1>(best, bi);
  dpp_argmax_step<0x4E>(best, bi);
  dpp_argmax_step<0x141>(best, bi);
  dpp_argmax_step<0x140>(best, bi);
  dpp_argmax_step<0x142, 0xA>(best, bi);
  dpp_argmax_step<0x143, 0xC>(best, bi);
}

// Sum over a workgroup of kThreads threads (4 waves); result valid in thread 0.
// Fixed shuffle tree, so the result is bitwise reproducible.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double *scratch /* [4*NV] shared */) {
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if (lane == 0) {
#pragma unroll
    for (int i = 0; i < NV; ++i) scratch[wid * NV + i] = v[i];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = (blockDim.x + 63) >> 6;
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      double s = scratch[i];
      for (int k = 1; k < nw; ++k) s += scratch[k * NV + i];
      v[i] = s;
    }
  }
  __syncthreads();
}

// Tile (gb, wb) of block `bid` in a 1-D launch over ngb x nwb tiles (ngb
// Cholesky-vector blocks, nwb walker blocks).  group == 0: gb fastest.
// group > 0: an order that keeps the operands of in-flight workgroups in each
// XCD's L2.  Workgroups are dealt to the 8 XCDs round-robin (XCD = bid mod 8),
// so each XCD is given one contiguous stretch of the tile order, and the order
// takes `group` walker blocks at a time across all Cholesky blocks, walker
// block fastest: a Cholesky tile is then read by `group` walker blocks while
// it is in L2, and their Theta stays resident.  Bijective for every size.
__device__ __forceinline__ void tile_of(int bid, int ntiles, int ngb, int nwb, int group, int &gb, int &wb) {
  if (group <= 0) {
    wb = bid / ngb;
    gb = bid - wb * ngb;
    return;
  }
  const int per = ntiles >> 3, rem = ntiles & 7;
  const int x = bid & 7, j = bid >> 3;
  const int t = x * per + min(x, rem) + j;
  const int span = group * ngb;
  const int g = t / span, within = t - g * span;
  const int gsize = min(group, nwb - g * group);
  wb = g * group + within % gsize;
  gb = within / gsize;
}

__device__ __forceinline__ double wrap_phase(double a) {
  const double twopi = 6.283185307179586476925286766559;
  double r = a - twopi * rint(a / twopi);
  if (r <= -3.14159265358979323846) r += twopi;
  return r;
}

// s_waitcnt that waits until at most n vector-memory operations of the wave are
// outstanding and leaves the LDS/scalar and export counters alone (gfx9
// encoding: vmcnt in bits 3:0 and 15:14, expcnt 6:4, lgkmcnt 11:8).
#define AFQMC_WAIT_VMCNT(n) __builtin_amdgcn_s_waitcnt(((n) & 15) | (7 << 4) | (15 << 8) | ((((n) >> 4) & 3) << 14))

}  // namespace afqmc
