// Reduced-precision forms of the exchange contraction (and of the force bias,
// which is its trace):
//   T^{g s}_w = Ltilde^{g s} Theta_{s,w},  EK = -1/2 sum_g sum_s Tr(T T),
//   vbias_g = sum_s Tr T^{g s}  (Sec. 2, eqs. Eloc and fb, by Wick's theorem).
// FP32 form: Ltilde and Theta rounded to FP32, v_mfma_f32_16x16x4f32, FP32
//   accumulation over the orbital index.
// Split-BF16 forms: every FP32 operand x is split into bfloat16 terms
//   x = h + m (+ l) (h = bf16(x), m = bf16(x - h), l = bf16(x - h - m)), and the
//   product is recovered on v_mfma_f32_16x16x32_bf16 with FP32 accumulation from
//   BF16x3: the six terms of order <= 2, hh + hm + mh + mm + hl + lh (the
//           dropped ml + lm + ll are below FP32 rounding);
//   BF16x2: the three terms hh + hm + mh (x is kept to about 2^-17 relative and
//           the dropped mm is of order 2^-18 of the product).
// In both forms T is kept in LDS as FP32; the FP32 form accumulates the traces in
// FP64, the split forms each lane's partial traces (at most 100 products) in FP32
// and the sums over lanes and Cholesky vectors in FP64.
// Overlaps, LU, propagation, weights and re-orthogonalisation stay FP64.
//
// Work decomposition as in the FP64 kernel: one GEMM per spin block with rows
// (g, i) padded to NR per Cholesky vector and columns (w, j, re/im) padded to
// CP = 2 NR per walker; wave (wy, wx) of a 2x2 grid owns GC whole Cholesky
// vectors and one whole walker.  MFMA lane layouts (gfx950, checked on the
// device): f32 16x16x4: lane l supplies A[l%16][l/16], B[l/16][l%16];
// bf16 16x16x32: lane l supplies A[l%16][8(l/16) .. 8(l/16)+7] and
// B[8(l/16) .. +7][l%16]; both: accumulator item r of lane l is
// D[4(l/16) + r][l%16].
#include <hip/hip_bf16.h>

#include "afqmc_internal.h"
#include "device_util.h"

namespace afqmc {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef __bf16 bf8v __attribute__((ext_vector_type(8)));

namespace {
constexpr int LWX = 2;      // walkers per workgroup
constexpr int LWY = 2;      // Cholesky-vector groups per workgroup
constexpr int LKC = 32;     // contraction rows per LDS stage
#ifndef AFQMC_EXCHANGE_DMA
#define AFQMC_EXCHANGE_DMA 1
#endif
constexpr bool kExchangeDma = AFQMC_EXCHANGE_DMA;  // stage the split-BF16 operands by LDS DMA
// Cholesky vectors per plane of the split-BF16 half rotation: G rounded up to
// whole workgroup rows (LWY groups of at most two vectors), the extra vectors
// zero, so every staged row a workgroup reads lies inside the planes.
__host__ __device__ constexpr int lp_padded_g(int G) { return (G + 2 * LWY - 1) / (2 * LWY) * (2 * LWY); }
}  // namespace

// Trace epilogue of the FP32 and three-term forms.  T of each wave (ROWW x CP
// floats) is in LDS at row stride TSF; every lane pairs each accumulator entry
// with the transposed entry of the same Cholesky vector and accumulates in R
// (FP64 or FP32).
template <int NR, int CT, int RT, typename R = double>
__device__ __forceinline__ void lp_trace(const f4v (&acc)[RT][CT], const float *sT, int TSF, int lane,
                                         R &pre, R &pim, R *dg) {
  const int lr = lane & 15, lk = lane >> 4;
  const bool odd = lr & 1;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int row = rt * 16 + 4 * lk + r;
        const int gl = row / NR, i = row - gl * NR;
        const int col = ct * 16 + lr, j = col >> 1;
        const float2 t = *reinterpret_cast<const float2 *>(sT + (gl * NR + j) * TSF + 2 * i);
        const R v = (R)acc[rt][ct][r];
        pre = fma(v, odd ? -(R)t.y : (R)t.x, pre);
        pim = fma(v, odd ? (R)t.x : (R)t.y, pim);
        const R d = (j == i) ? v : (R)0;
        if (gl == 0) dg[0] += d;
        else dg[1] += d;
      }
}

// Trace epilogue of the two-term form, one Cholesky vector (pass) of the wave
// at a time.  T^g goes to LDS as two planes, Re and Im, of U[j][i] = T^g_ij at
// row stride NR + 4: a lane's four accumulator rows i0..i0+3 of column (j, re|im)
// are one 16-byte store, and the partner T^g_ji of an entry is two 4-byte reads
// at offsets fixed at compile time, so the epilogue is almost free of VALU work
// (a wave64 VALU instruction costs four cycles of the SIMD).  Rows of one tile
// belong to one Cholesky vector unless the tile straddles two (NR % 16 != 0);
// in that tile each lane's four rows still share one.
template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_store_u(const f4v (&acc)[RT][CT], float *sU, int lane, int pass) {
  constexpr int CS = NR + 4;
  const int lr = lane & 15, lk = lane >> 4;
  const int sidx = (lr & 1) * NR * CS + (lr >> 1) * CS + 4 * lk - pass * NR;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    const bool mine = glo == ghi || (rt * 16 + 4 * lk) / NR == pass;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
      if (mine) *reinterpret_cast<f4v *>(sU + sidx + ct * 8 * CS + rt * 16) = acc[rt][ct];
  }
}

template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_trace_u(const f4v (&acc)[RT][CT], const float *sU, int lane, float &pre,
                                           float &pim, float *dg, int pass) {
  constexpr int CS = NR + 4;
  const int lr = lane & 15, lk = lane >> 4;
  const bool odd = lr & 1;
  const int bidx = (4 * lk - pass * NR) * CS + (lr >> 1);   // + (rt 16 + r) CS + 8 ct: U[i][j], row i of the pass
  float a0 = 0.f, a1 = 0.f;                                 // sum of v Re T_ji, sum of v Im T_ji
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    const bool mine = glo == ghi || (rt * 16 + 4 * lk) / NR == pass;
    if (!mine) continue;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int off = bidx + (rt * 16 + r) * CS + ct * 8;
        const float v = acc[rt][ct][r];
        a0 = fmaf(v, sU[off], a0);
        a1 = fmaf(v, sU[NR * CS + off], a1);
      }
  }
  // the lane holds Re T_ij (even lr) or Im T_ij (odd lr)
  pre += odd ? -a1 : a0;
  pim += odd ? a0 : a1;
  // diagonal, in the parity convention of lp_finish: lane l adds Re (l even)
  // or Im (l odd) of T_ii, i = l / 2
  for (int l = lane; l < 2 * NR; l += 64) {
    const int i = l >> 1;
    dg[pass] += sU[(l & 1) * NR * CS + i * CS + i];
  }
}

template <int GC>
__device__ __forceinline__ void lp_finish(double pre, double pim, const double *dg, int lane, int w, int W, int g0w,
                                          int G, int spin, int stride, int part, double2 *ekpart,
                                          double2 *vbpart) {
  pre = wave_sum_dpp(pre);
  pim = wave_sum_dpp(pim);
  if (lane == 63 && w < W && g0w < G)
    ekpart[((size_t)w * 2 + spin) * stride + part] = make_double2(-0.5 * pre, -0.5 * pim);
  if (vbpart) {
    const bool odd = lane & 1;
#pragma unroll
    for (int gl = 0; gl < GC; ++gl) {
      double dre = odd ? 0.0 : dg[gl], dim = odd ? dg[gl] : 0.0;
      dre = wave_sum_dpp(dre);
      dim = wave_sum_dpp(dim);
      const int g = g0w + gl;
      if (lane == 63 && w < W && g < G) vbpart[((size_t)spin * W + w) * G + g] = make_double2(dre, dim);
    }
  }
}

// ---- FP32 form ----------------------------------------------------------------
// LtF[g][q][NR] (float, padded rows), ThF[w][q][CP] (float, interleaved complex,
// padded columns) for one spin block.
template <int NR>
__global__ __launch_bounds__(kThreads) void k_exchange_f32(const float *__restrict__ LtF,
                                                          const float *__restrict__ ThF, int M, int N, int G, int W,
                                                          int stride, int spin, double2 *__restrict__ ekpart,
                                                          double2 *__restrict__ vbpart, int ngb, int nwb,
                                                          int group) {
  constexpr int GC = (NR % 16 == 0) ? 1 : 2;
  constexpr int ROWW = GC * NR, RT = ROWW / 16;
  constexpr int CP = 2 * NR, CT = CP / 16;
  constexpr int ROWS = LWY * ROWW;
  constexpr int ASZ = LKC * ROWS, BSZ = LWX * LKC * CP;          // floats per stage
  constexpr int APT = (ASZ / 4 + kThreads - 1) / kThreads;      // float4 loads per thread
  constexpr int BPT = (BSZ / 4 + kThreads - 1) / kThreads;
  constexpr int TSF = CP + 2;
  extern __shared__ float fsm[];
  float *sA = fsm, *sB = fsm + 2 * ASZ;

  int gb, wb;
  tile_of(blockIdx.x, ngb * nwb, ngb, nwb, group, gb, wb);
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int wy = wv / LWX, wx = wv - (wv / LWX) * LWX;
  const int g0 = gb * LWY * GC, w0 = wb * LWX;

  float4 ra[APT], rb[BPT];
  auto load = [&](int q0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int e = 4 * (tid + r * kThreads);
      const int q = e / ROWS, row = e - q * ROWS;
      const int gl = row / NR, i = row - gl * NR;
      const int g = g0 + gl, gq = q0 + q;
      ra[r] = (e < ASZ && g < G && gq < M) ? *reinterpret_cast<const float4 *>(LtF + ((size_t)g * M + gq) * NR + i)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int e = 4 * (tid + r * kThreads);
      const int c = e % CP, t = e / CP;
      const int q = t % LKC, wl = t / LKC;
      const int w = w0 + wl, gq = q0 + q;
      rb[r] = (e < BSZ && w < W && gq < M) ? *reinterpret_cast<const float4 *>(ThF + ((size_t)w * M + gq) * CP + c)
                                          : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store = [&](int buf) {
    float4 *a = reinterpret_cast<float4 *>(sA + buf * ASZ);
    float4 *b = reinterpret_cast<float4 *>(sB + buf * BSZ);
#pragma unroll
    for (int r = 0; r < APT; ++r)
      if (4 * (tid + r * kThreads) < ASZ) a[tid + r * kThreads] = ra[r];
#pragma unroll
    for (int r = 0; r < BPT; ++r)
      if (4 * (tid + r * kThreads) < BSZ) b[tid + r * kThreads] = rb[r];
  };

  f4v acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  const int nchunk = (M + LKC - 1) / LKC;
  load(0);
  store(0);
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch & 1;
    if (ch + 1 < nchunk) load((ch + 1) * LKC);
    const float *a = sA + buf * ASZ + wy * ROWW + lr;
    const float *b = sB + buf * BSZ + wx * LKC * CP + lr;
#pragma unroll
    for (int ks = 0; ks < LKC / 4; ++ks) {
      float av[RT], bv[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) av[i] = a[(ks * 4 + lk) * ROWS + i * 16];
#pragma unroll
      for (int j = 0; j < CT; ++j) bv[j] = b[(ks * 4 + lk) * CP + j * 16];
#pragma unroll
      for (int i = 0; i < RT; ++i)
#pragma unroll
        for (int j = 0; j < CT; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x4f32(av[i], bv[j], acc[i][j], 0, 0, 0);
    }
    if (ch + 1 < nchunk) store(buf ^ 1);
    __syncthreads();
  }

  float *sT = fsm + (size_t)wv * ROWW * TSF;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt)
#pragma unroll
    for (int ct = 0; ct < CT; ++ct)
#pragma unroll
      for (int r = 0; r < 4; ++r) sT[(rt * 16 + 4 * lk + r) * TSF + ct * 16 + lr] = acc[rt][ct][r];
  __syncthreads();
  double pre = 0.0, pim = 0.0, dg[2] = {0.0, 0.0};
  lp_trace<NR, CT, RT>(acc, sT, TSF, lane, pre, pim, dg);
  lp_finish<GC>(pre, pim, dg, lane, w0 + wx, W, g0 + wy * GC, G, spin, stride, gb * LWY + wy, ekpart, vbpart);
}

// ---- split-BF16 forms ----------------------------------------------------------
// LtB[p][g][NR][Kp] (g over lp_padded_g(G), the extra vectors zero),
// ThB[p][w][CP][Kp] (bf16, p = h, m (, l) for NT = 2 (3) terms; contraction
// index contiguous and zero-padded to Kp, a multiple of 32) for one spin block.
template <int NR, int NT>
__global__ __launch_bounds__(kThreads, NT == 2 ? 2 : 1) void k_exchange_bf16(const __bf16 *__restrict__ LtB,
                                                             const __bf16 *__restrict__ ThB, int Kp, int N, int G,
                                                             int W, int stride, int spin,
                                                             double2 *__restrict__ ekpart,
                                                             double2 *__restrict__ vbpart, int ngb, int nwb,
                                                             int group) {
  constexpr int GC = (NR % 16 == 0) ? 1 : 2;
  constexpr int ROWW = GC * NR, RT = ROWW / 16;
  constexpr int CP = 2 * NR, CT = CP / 16;
  constexpr int ROWS = LWY * ROWW;
  constexpr int COLS = LWX * CP;
  // Staged rows are LKC = 32 bf16 (64 bytes) with no padding; the four 16-byte
  // k groups of row r sit in slots k8 ^ swz(r), so the 16 rows one MFMA operand
  // read touches at one k group fall in distinct banks, and a row is still one
  // 64-byte run for the stores.
  constexpr int RS = LKC;                        // staged row stride (bf16)
  constexpr int ASZ = NT * ROWS * RS, BSZ = NT * COLS * RS;   // bf16 per stage
  constexpr int AV = NT * ROWS * (LKC / 8), BV = NT * COLS * (LKC / 8);  // 16-byte vectors per stage
  constexpr int APT = (AV + kThreads - 1) / kThreads, BPT = (BV + kThreads - 1) / kThreads;
  constexpr int TSF = CP + 2;
  static_assert(ROWW % 16 == 0 && CP % 16 == 0 && LKC == 32, "row bases keep the swizzle of the lane's row");
  // Two staging buffers (one barrier per chunk).  The two-term form fits two
  // workgroups per CU (80 KB of LDS, registers for two waves per SIMD) and does
  // the trace epilogue one Cholesky vector of each wave at a time.
  constexpr int NBUF = 2;
  auto swz = [](int r) { return ((r >> 1) ^ (r >> 2)) & 3; };
  extern __shared__ __bf16 bsm[];
  __bf16 *sA = bsm, *sB = bsm + NBUF * ASZ;
  // With LDS DMA (global_load_lds_dwordx4: lane L's 16 bytes land at the wave's
  // LDS base + 16 L) a stage is filled straight from memory, 1 KB (16 staged
  // rows) per wave instruction (sources below).
  constexpr bool DMA = kExchangeDma;
  static_assert(AV % 64 == 0 && BV % 64 == 0, "whole 1 KB blocks");

  int gb, wb;
  tile_of(blockIdx.x, ngb * nwb, ngb, nwb, group, gb, wb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: LDS stage addresses stay scalar
  const int wy = wv / LWX, wx = wv - (wv / LWX) * LWX;
  const int g0 = gb * LWY * GC, w0 = wb * LWX;
  const size_t aplane = (size_t)lp_padded_g(G) * NR * Kp, bplane = (size_t)W * CP * Kp;

  uint4 ra[APT], rb[BPT];
  auto load = [&](int q0) {
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int v = tid + r * kThreads;                  // (p, row, k8)
      const int k8 = v % (LKC / 8), t = v / (LKC / 8);
      const int row = t % ROWS, p = t / ROWS;
      const int gl = row / NR, i = row - gl * NR, g = g0 + gl;
      ra[r] = (v < AV && g < G)
                  ? *reinterpret_cast<const uint4 *>(LtB + p * aplane + ((size_t)g * NR + i) * Kp + q0 + 8 * k8)
                  : make_uint4(0u, 0u, 0u, 0u);
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int v = tid + r * kThreads;                  // (p, col, k8)
      const int k8 = v % (LKC / 8), t = v / (LKC / 8);
      const int col = t % COLS, p = t / COLS;
      const int wl = col / CP, c = col - wl * CP, w = w0 + wl;
      rb[r] = (v < BV && w < W)
                  ? *reinterpret_cast<const uint4 *>(ThB + p * bplane + ((size_t)w * CP + c) * Kp + q0 + 8 * k8)
                  : make_uint4(0u, 0u, 0u, 0u);
    }
  };
  auto store = [&](int buf) {
    __bf16 *a = sA + buf * ASZ;
    __bf16 *b = sB + buf * BSZ;
#pragma unroll
    for (int r = 0; r < APT; ++r) {
      const int v = tid + r * kThreads;
      if (v < AV) {
        const int k8 = v % (LKC / 8), t = v / (LKC / 8);
        *reinterpret_cast<uint4 *>(a + t * RS + 8 * (k8 ^ swz(t))) = ra[r];
      }
    }
#pragma unroll
    for (int r = 0; r < BPT; ++r) {
      const int v = tid + r * kThreads;
      if (v < BV) {
        const int k8 = v % (LKC / 8), t = v / (LKC / 8);
        *reinterpret_cast<uint4 *>(b + t * RS + 8 * (k8 ^ swz(t))) = rb[r];
      }
    }
  };

  // LDS DMA sources: this lane's 16 bytes of every staged row it fills, as
  // element offsets at k = 0 (loop-invariant; a chunk adds q0 to the uniform
  // base).  Rows past G are the zero vectors of the padded planes; columns of
  // walkers past W repeat walker W - 1 (their results are never written).
  constexpr int NIA = (AV / 64 + 3) / 4, NIB = (BV / 64 + 3) / 4;
  uint32_t offa[NIA], offb[NIB];
  {
    const int t4 = lane >> 2, slot = lane & 3;
#pragma unroll
    for (int r = 0; r < NIA; ++r) {
      const int blk = wv + 4 * r, t = 16 * blk + t4;          // staged row (p, row)
      const int row = t % ROWS, p = t / ROWS;
      const int gl = row / NR, i = row - gl * NR, g = g0 + gl;
      offa[r] = (uint32_t)(p * aplane + ((size_t)g * NR + i) * Kp + 8 * (slot ^ swz(t)));
    }
#pragma unroll
    for (int r = 0; r < NIB; ++r) {
      const int blk = wv + 4 * r, t = 16 * blk + t4;          // staged column (p, col)
      const int col = t % COLS, p = t / COLS;
      const int wl = col / CP, c = col - wl * CP, w = min(w0 + wl, W - 1);
      offb[r] = (uint32_t)(p * bplane + ((size_t)w * CP + c) * Kp + 8 * (slot ^ swz(t)));
    }
  }
  auto issue = [&](int q0, int buf) {
    __bf16 *a = sA + buf * ASZ;
    __bf16 *b = sB + buf * BSZ;
    const __bf16 *la = LtB + q0, *tb = ThB + q0;
#pragma unroll
    for (int r = 0; r < NIA; ++r) {
      const int blk = wv + 4 * r;
      if ((AV / 64) % 4 != 0 && blk >= AV / 64) break;       // uniform in the wave
      const __bf16 *src = la + offa[r];
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(a + blk * 512), 16, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < NIB; ++r) {
      const int blk = wv + 4 * r;
      if ((BV / 64) % 4 != 0 && blk >= BV / 64) break;       // uniform in the wave
      const __bf16 *src = tb + offb[r];
      __builtin_amdgcn_global_load_lds(src, (__attribute__((address_space(3))) void *)(b + blk * 512), 16, 0, 0);
    }
  };

  f4v acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  const int nchunk = Kp / LKC;
  if constexpr (DMA) {
    issue(0, 0);
    __builtin_amdgcn_s_waitcnt(0);
  } else {
    load(0);
    store(0);
  }
  __syncthreads();
  const int lr = lane & 15, lk = lane >> 4;
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = NBUF == 2 ? (ch & 1) : 0;
    if constexpr (DMA) {
      if (ch + 1 < nchunk) issue((ch + 1) * LKC, buf ^ 1);
    } else if (ch + 1 < nchunk) {
      load((ch + 1) * LKC);
    }
    const __bf16 *a = sA + buf * ASZ + (wy * ROWW + lr) * RS + 8 * (lk ^ swz(lr));
    const __bf16 *b = sB + buf * BSZ + (wx * CP + lr) * RS + 8 * (lk ^ swz(lr));
    bf8v ah[RT], am[RT], bh[CT], bm[CT];
    // the fragments of the first sweep (am x bh) are read first; the other
    // RT + CT reads are spread over that sweep's MFMAs (the group barriers
    // below), so an MFMA waits only on the reads it uses
#pragma unroll
    for (int i = 0; i < (RT > CT ? RT : CT); ++i) {
      if (i < RT) am[i] = *reinterpret_cast<const bf8v *>(a + (1 * ROWS + i * 16) * RS);
      if (i < CT) bh[i] = *reinterpret_cast<const bf8v *>(b + (0 * COLS + i * 16) * RS);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < CT; ++j) bm[j] = *reinterpret_cast<const bf8v *>(b + (1 * COLS + j * 16) * RS);
#pragma unroll
    for (int i = 0; i < RT; ++i) ah[i] = *reinterpret_cast<const bf8v *>(a + (0 * ROWS + i * 16) * RS);
    // one sweep over all accumulators per term, so dependent MFMAs are far
    // apart; the smallest terms first
#define AFQMC_SWEEP(X, Y)                                                                         \
  _Pragma("unroll") for (int i = 0; i < RT; ++i) _Pragma("unroll") for (int j = 0; j < CT; ++j) \
      acc[i][j] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(X[i], Y[j], acc[i][j], 0, 0, 0);
    if constexpr (NT == 3) {
      bf8v al[RT], bl[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) al[i] = *reinterpret_cast<const bf8v *>(a + (2 * ROWS + i * 16) * RS);
#pragma unroll
      for (int j = 0; j < CT; ++j) bl[j] = *reinterpret_cast<const bf8v *>(b + (2 * COLS + j * 16) * RS);
      AFQMC_SWEEP(al, bh)
      AFQMC_SWEEP(ah, bl)
      AFQMC_SWEEP(am, bm)
    }
    AFQMC_SWEEP(am, bh)
    AFQMC_SWEEP(ah, bm)
    AFQMC_SWEEP(ah, bh)
#undef AFQMC_SWEEP
    if constexpr (NT == 2 && 3 * RT * CT > 2 * (RT + CT)) {
#pragma unroll
      for (int q = 0; q < RT + CT; ++q) {
        __builtin_amdgcn_sched_group_barrier(0x008, 2, 0);   // two MFMAs
        __builtin_amdgcn_sched_group_barrier(0x100, 1, 0);   // one LDS read
      }
      __builtin_amdgcn_sched_group_barrier(0x008, 3 * RT * CT - 2 * (RT + CT), 0);
    }
    // keep every MFMA of the chunk ahead of the wait for the next stage (the
    // scheduler would otherwise sink most of them below the barrier, leaving
    // the copies a fraction of the chunk to land in)
    __builtin_amdgcn_sched_barrier(0);
    if constexpr (DMA) {
      __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into the other buffer have landed
    } else if (ch + 1 < nchunk) {
      store(buf ^ 1);
    }
    __syncthreads();
  }

  // each lane's partial traces (at most ROWW CP / 64 products) in FP32, the
  // sums over lanes and Cholesky vectors in FP64
  float pre = 0.f, pim = 0.f, dg[2] = {0.f, 0.f};
  if constexpr (NT == 2) {
    // one Cholesky vector of the wave at a time: U (two NR x (NR + 4) planes) per wave in LDS
    float *sU = reinterpret_cast<float *>(bsm) + (size_t)wv * NR * (NR + 4) * 2;
#pragma unroll
    for (int pass = 0; pass < GC; ++pass) {
      lp_store_u<NR, CT, RT>(acc, sU, lane, pass);
      __syncthreads();
      lp_trace_u<NR, CT, RT>(acc, sU, lane, pre, pim, dg, pass);
      if (pass + 1 < GC) __syncthreads();
    }
  } else {
    float *sT = reinterpret_cast<float *>(bsm) + (size_t)wv * ROWW * TSF;
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) sT[(rt * 16 + 4 * lk + r) * TSF + ct * 16 + lr] = acc[rt][ct][r];
    __syncthreads();
    lp_trace<NR, CT, RT, float>(acc, sT, TSF, lane, pre, pim, dg);
  }
  const double dgd[2] = {(double)dg[0], (double)dg[1]};
  lp_finish<GC>((double)pre, (double)pim, dgd, lane, w0 + wx, W, g0 + wy * GC, G, spin, stride, gb * LWY + wy, ekpart,
                vbpart);
}

// ---- operand preparation -------------------------------------------------------
__device__ __forceinline__ void split3(float x, __bf16 &h, __bf16 &m, __bf16 &l) {
  h = (__bf16)x;
  const float r1 = x - (float)h;
  m = (__bf16)r1;
  l = (__bf16)(r1 - (float)m);
}

// LtF[g][q][i] = float(LtS[g][q][i])
__global__ void k_lt_to_f32(const double *__restrict__ LtS, long n, float *__restrict__ LtF) {
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e < n) LtF[e] = (float)LtS[e];
}

// LtB[p][g][i][q] (p < NT) from LtS[g][q][i] (rows i < NR, q < Kp, zero for q >= M)
template <int NT>
__global__ void k_lt_to_bf16(const double *__restrict__ LtS, int G, int M, int NR, int Kp, __bf16 *__restrict__ LtB) {
  const long n = (long)lp_padded_g(G) * NR * Kp;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int q = (int)(e % Kp);
  const long t = e / Kp;
  const int i = (int)(t % NR);
  const int g = (int)(t / NR);
  const float x = (q < M && g < G) ? (float)LtS[((size_t)g * M + q) * NR + i] : 0.f;
  __bf16 h, m, l;
  split3(x, h, m, l);
  LtB[e] = h;
  LtB[n + e] = m;
  if (NT == 3) LtB[2 * n + e] = l;
}

// ThF[w][q][c] (c < CP) from Theta[w][q][off + c/2] (re/im by parity), zero-padded
__global__ void k_theta_to_f32(const double2 *__restrict__ theta, int W, int M, int Nt, int off, int N, int CP,
                               float *__restrict__ ThF) {
  const long n = (long)W * M * CP;
  const long e = (long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= n) return;
  const int c = (int)(e % CP);
  const long wq = e / CP;
  float v = 0.f;
  if (c < 2 * N) {
    const double2 z = theta[(size_t)wq * Nt + off + (c >> 1)];
    v = (float)((c & 1) ? z.y : z.x);
  }
  ThF[e] = v;
}

// ThB[p][w][c][q] (p < NT, q < Kp) from Theta[w][q][off + c/2]; one workgroup
// per (walker, 32 rows q) transposes through LDS
template <int NT>
__global__ __launch_bounds__(kThreads) void k_theta_to_bf16(const double2 *__restrict__ theta, int W, int M, int Nt,
                                                             int off, int N, int CP, int Kp,
                                                             __bf16 *__restrict__ ThB) {
  extern __shared__ float tsm[];  // [32][CP + 1]
  const int w = blockIdx.y, q0 = blockIdx.x * 32;
  const int tid = threadIdx.x;
  for (int e = tid; e < 32 * CP; e += blockDim.x) {
    const int qq = e / CP, c = e - qq * CP;
    const int q = q0 + qq;
    float v = 0.f;
    if (q < M && c < 2 * N) {
      const double2 z = theta[((size_t)w * M + q) * Nt + off + (c >> 1)];
      v = (float)((c & 1) ? z.y : z.x);
    }
    tsm[qq * (CP + 1) + c] = v;
  }
  __syncthreads();
  const size_t plane = (size_t)W * CP * Kp;
  for (int e = tid; e < 32 * CP; e += blockDim.x) {
    const int c = e / 32, qq = e - c * 32;
    __bf16 h, m, l;
    split3(tsm[qq * (CP + 1) + c], h, m, l);
    const size_t o = ((size_t)w * CP + c) * Kp + q0 + qq;
    ThB[o] = h;
    ThB[plane + o] = m;
    if (NT == 3) ThB[2 * plane + o] = l;
  }
}

// ---- dispatch -------------------------------------------------------------------
namespace {
using F32Kernel = void (*)(const float *, const float *, int, int, int, int, int, int, double2 *, double2 *, int,
                           int, int);
using BFKernel = void (*)(const __bf16 *, const __bf16 *, int, int, int, int, int, int, double2 *, double2 *, int,
                          int, int);

F32Kernel pick_f32(int nr) {
  switch (nr) {
    case 8: return k_exchange_f32<8>;
    case 16: return k_exchange_f32<16>;
    case 24: return k_exchange_f32<24>;
    case 32: return k_exchange_f32<32>;
    case 40: return k_exchange_f32<40>;
    case 48: return k_exchange_f32<48>;
    default: return nullptr;
  }
}
template <int NT>
BFKernel pick_bf_nt(int nr) {
  switch (nr) {
    case 8: return k_exchange_bf16<8, NT>;
    case 16: return k_exchange_bf16<16, NT>;
    case 24: return k_exchange_bf16<24, NT>;
    case 32: return k_exchange_bf16<32, NT>;
    case 40: return k_exchange_bf16<40, NT>;
    case 48: return k_exchange_bf16<48, NT>;
    default: return nullptr;
  }
}
// bfloat16 terms per operand of a split-BF16 precision (0: not a split form)
int bf_terms(int precision) {
  return precision == AFQMC_BF16X3_CONTRACT ? 3 : precision == AFQMC_BF16X2_CONTRACT ? 2 : 0;
}
BFKernel pick_bf(int nr, int nt) { return nt == 3 ? pick_bf_nt<3>(nr) : nt == 2 ? pick_bf_nt<2>(nr) : nullptr; }
size_t lds_f32(int nr) {
  const int gc = (nr % 16 == 0) ? 1 : 2, roww = gc * nr, cp = 2 * nr;
  const size_t stage = 2ull * (LKC * LWY * roww + LWX * LKC * cp) * sizeof(float);
  const size_t epi = 4ull * roww * (cp + 2) * sizeof(float);
  return stage > epi ? stage : epi;
}
size_t lds_bf(int nr, int nt) {
  const int gc = (nr % 16 == 0) ? 1 : 2, roww = gc * nr, cp = 2 * nr;
  const size_t nbuf = 2;
  const size_t stage = nbuf * nt * (LWY * roww + LWX * cp) * LKC * sizeof(__bf16);
  const size_t epi = nt == 2 ? 4ull * nr * (nr + 4) * 2 * sizeof(float) : 4ull * roww * (cp + 2) * sizeof(float);
  return stage > epi ? stage : epi;
}
}  // namespace

bool lp_exchange_supported(int precision, int nr) {
  if (precision == AFQMC_FP32_CONTRACT) return pick_f32(nr) && lds_f32(nr) <= 160 * 1024;
  const int nt = bf_terms(precision);
  if (nt) return pick_bf(nr, nt) && lds_bf(nr, nt) <= 160 * 1024;
  return false;
}

size_t lp_operand_elems(int precision, int G, int M, int W, int nr, bool lhs) {
  const int kp = ((M + LKC - 1) / LKC) * LKC;
  if (precision == AFQMC_FP32_CONTRACT) return lhs ? (size_t)G * M * nr : (size_t)W * M * 2 * nr;
  const size_t nt = bf_terms(precision);
  return lhs ? nt * lp_padded_g(G) * nr * kp : nt * W * 2 * nr * kp;
}

bool lp_operands_addressable(int precision, int G, int M, int W, int nr) {
  if (!bf_terms(precision)) return true;
  const size_t lim = (size_t)1 << 32;
  return lp_operand_elems(precision, G, M, W, nr, true) < lim && lp_operand_elems(precision, G, M, W, nr, false) < lim;
}

hipError_t lp_prepare_lhs(const System &s, int spin, hipStream_t st) {
  const ExchangePlan &p = s.ex_plan[spin];
  if (p.N == 0) return hipSuccess;
  if (s.precision == AFQMC_FP32_CONTRACT) {
    const long n = (long)s.G * s.M * p.NR;
    hipLaunchKernelGGL(k_lt_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.LtS[spin], n,
                       static_cast<float *>(s.lp_lhs[spin]));
  } else {
    const int kp = ((s.M + LKC - 1) / LKC) * LKC;
    const long n = (long)lp_padded_g(s.G) * p.NR * kp;
    hipLaunchKernelGGL(bf_terms(s.precision) == 3 ? k_lt_to_bf16<3> : k_lt_to_bf16<2>,
                       dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, s.LtS[spin], s.G, s.M, p.NR, kp,
                       static_cast<__bf16 *>(s.lp_lhs[spin]));
  }
  return hipGetLastError();
}

hipError_t lp_enable_lds(const System &s) {
  for (int spin = 0; spin < 2; ++spin) {
    const ExchangePlan &p = s.ex_plan[spin];
    if (p.N == 0) continue;
    hipError_t e = hipSuccess;
    if (s.precision == AFQMC_FP32_CONTRACT)
      e = hipFuncSetAttribute(reinterpret_cast<const void *>(pick_f32(p.NR)),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_f32(p.NR));
    else
      e = hipFuncSetAttribute(reinterpret_cast<const void *>(pick_bf(p.NR, bf_terms(s.precision))),
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds_bf(p.NR, bf_terms(s.precision)));
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

hipError_t lp_prepare_rhs(const System &s, const double2 *theta, int W, int spin, hipStream_t st) {
  const ExchangePlan &p = s.ex_plan[spin];
  if (p.N == 0) return hipSuccess;
  const int off = spin ? s.Na : 0;
  const int CP = 2 * p.NR;
  if (s.precision == AFQMC_FP32_CONTRACT) {
    const long n = (long)W * s.M * CP;
    hipLaunchKernelGGL(k_theta_to_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, st, theta, W, s.M, s.Nt,
                       off, p.N, CP, static_cast<float *>(s.lp_rhs[spin]));
  } else {
    const int kp = ((s.M + LKC - 1) / LKC) * LKC;
    hipLaunchKernelGGL(bf_terms(s.precision) == 3 ? k_theta_to_bf16<3> : k_theta_to_bf16<2>, dim3(kp / 32, W),
                       dim3(kThreads), 32 * (CP + 1) * sizeof(float), st, theta, W, s.M, s.Nt, off, p.N, CP, kp,
                       static_cast<__bf16 *>(s.lp_rhs[spin]));
  }
  return hipGetLastError();
}

hipError_t launch_exchange_lp(const System &s, int W, int spin, hipStream_t st, double2 *vbpart) {
  const ExchangePlan &p = s.ex_plan[spin];
  if (p.N == 0) return vbpart ? launch_zero2(vbpart + (size_t)spin * W * s.G, (long)W * s.G, st) : hipSuccess;
  const int gc = p.GC;
  const int ngb = (s.G + LWY * gc - 1) / (LWY * gc), nwb = (W + LWX - 1) / LWX;
  const dim3 grid((unsigned)(ngb * nwb));
  if (s.precision == AFQMC_FP32_CONTRACT) {
    hipLaunchKernelGGL(pick_f32(p.NR), grid, dim3(kThreads), lds_f32(p.NR), st,
                       static_cast<const float *>(s.lp_lhs[spin]), static_cast<const float *>(s.lp_rhs[spin]), s.M,
                       p.N, s.G, W, s.ex_stride, spin, s.ekpart, vbpart, ngb, nwb, s.ex_group);
  } else {
    const int kp = ((s.M + LKC - 1) / LKC) * LKC;
    const int nt = bf_terms(s.precision);
    hipLaunchKernelGGL(pick_bf(p.NR, nt), grid, dim3(kThreads), lds_bf(p.NR, nt), st,
                       static_cast<const __bf16 *>(s.lp_lhs[spin]), static_cast<const __bf16 *>(s.lp_rhs[spin]), kp,
                       p.N, s.G, W, s.ex_stride, spin, s.ekpart, vbpart, ngb, nwb, s.ex_group);
  }
  return hipGetLastError();
}

}  // namespace afqmc
