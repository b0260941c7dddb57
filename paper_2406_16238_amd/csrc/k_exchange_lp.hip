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
// Trial-split forms (FP16 or BF16, one product): Theta = Psi + Q with Psi^T Q = 0
//   (Psi^T Theta = 1), so T = T0 + Ltilde Q with T0 = Ltilde Psi fixed at set-up
//   (FP32) and only the walker's departure Q from the trial rounded: Ltilde^g and
//   Q_w are scaled by powers of two (per Cholesky vector, per walker) into one
//   16-bit term each, multiplied on v_mfma_f32_16x16x32_{f16,bf16} with FP32
//   accumulation; the accumulators start at T0 divided by the two scales and
//   the epilogue multiplies them back.  The rounding error of the 16-bit terms
//   is relative to Ltilde Q, not to T.
// In all forms T is kept in LDS as FP32; the FP32 form accumulates the traces in
// FP64, the 16-bit forms each lane's partial traces (at most 100 products) in
// FP32 and the sums over lanes and Cholesky vectors in FP64.
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
typedef _Float16 h8v __attribute__((ext_vector_type(8)));

// 8-wide operand vector of a 16-bit element type, and the 16x16x32 MFMA on it
template <typename E> struct Vec8;
template <> struct Vec8<__bf16> { typedef bf8v type; };
template <> struct Vec8<_Float16> { typedef h8v type; };
__device__ __forceinline__ f4v mfma16x16x32(bf8v a, bf8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}
__device__ __forceinline__ f4v mfma16x16x32(h8v a, h8v b, f4v c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_f16(a, b, c, 0, 0, 0);
}

namespace {
constexpr int LWX = 2;      // walkers per workgroup
constexpr int LWY = 2;      // Cholesky-vector groups per workgroup
constexpr int LKC = 32;     // contraction rows per LDS stage
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

// Trace epilogue of the 16-bit forms, one Cholesky vector (pass) of the wave at
// a time, through LDS in natural order: S[i][j] = T_ij as two planes, Re and Im,
// at row stride NR + 4, the Im plane 8 words past the Re plane (so the 64 lanes
// of one store fall into distinct banks).  A lane stores its four accumulator
// rows of column (j, re|im) as four words, and reads the partners T_ji of those
// rows, T_{j, i0..i0+3}, as one 16-byte word per plane.  The waves use disjoint
// LDS and exchange nothing, so no barrier is needed between store and read.
template <int NR>
__host__ __device__ constexpr int lp_s_plane() { return NR * (NR + 4) + 8; }

template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_store_s(const f4v (&acc)[RT][CT], float *sS, int lane, int pass) {
  constexpr int CS = NR + 4, PL = lp_s_plane<NR>();
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    if ((rt * 16 + 4 * lk) / NR != pass) continue;   // the lane's four rows belong to one Cholesky vector
    const int i0 = rt * 16 + 4 * lk - pass * NR;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      float *d = sS + (lr & 1) * PL + i0 * CS + ct * 8 + (lr >> 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) d[r * CS] = acc[rt][ct][r];
    }
  }
}

template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_trace_s(const f4v (&acc)[RT][CT], const float *sS, int lane, float &pre,
                                           float &pim, int pass) {
  constexpr int CS = NR + 4, PL = lp_s_plane<NR>();
  const int lr = lane & 15, lk = lane >> 4;
  const bool odd = lr & 1;
  float a0 = 0.f, a1 = 0.f;   // sum v Re T_ji, sum v Im T_ji
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    if ((rt * 16 + 4 * lk) / NR != pass) continue;
    const int i0 = rt * 16 + 4 * lk - pass * NR;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int j = ct * 8 + (lr >> 1);
      const f4v cre = *reinterpret_cast<const f4v *>(sS + j * CS + i0);
      const f4v cim = *reinterpret_cast<const f4v *>(sS + PL + j * CS + i0);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const float v = acc[rt][ct][r];
        a0 = fmaf(v, cre[r], a0);
        a1 = fmaf(v, cim[r], a1);
      }
    }
  }
  // the lane holds Re T_ij (even lr) or Im T_ij (odd lr)
  pre += odd ? -a1 : a0;
  pim += odd ? a0 : a1;
}

// The same trace with one plane of S in LDS at a time (half the LDS): the
// lanes holding Re T_ij (part 0, even lr) or Im T_ij (part 1) store their
// entries, then every lane reads the partners from that plane.
template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_store_s1(const f4v (&acc)[RT][CT], float *sS, int lane, int pass, int part) {
  constexpr int CS = NR + 4;
  const int lr = lane & 15, lk = lane >> 4;
  if ((lr & 1) != part) return;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    if ((rt * 16 + 4 * lk) / NR != pass) continue;   // the lane's four rows belong to one Cholesky vector
    const int i0 = rt * 16 + 4 * lk - pass * NR;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      float *d = sS + i0 * CS + ct * 8 + (lr >> 1);
#pragma unroll
      for (int r = 0; r < 4; ++r) d[r * CS] = acc[rt][ct][r];
    }
  }
}

// a += sum v * (plane entry of the partner T_ji)
template <int NR, int CT, int RT>
__device__ __forceinline__ void lp_trace_s1(const f4v (&acc)[RT][CT], const float *sS, int lane, float &a, int pass) {
  constexpr int CS = NR + 4;
  const int lr = lane & 15, lk = lane >> 4;
#pragma unroll
  for (int rt = 0; rt < RT; ++rt) {
    const int glo = rt * 16 / NR, ghi = (rt * 16 + 15) / NR;
    if (glo == ghi && glo != pass) continue;
    if ((rt * 16 + 4 * lk) / NR != pass) continue;
    const int i0 = rt * 16 + 4 * lk - pass * NR;
#pragma unroll
    for (int ct = 0; ct < CT; ++ct) {
      const int j = ct * 8 + (lr >> 1);
      const f4v c = *reinterpret_cast<const f4v *>(sS + j * CS + i0);
#pragma unroll
      for (int r = 0; r < 4; ++r) a = fmaf(acc[rt][ct][r], c[r], a);
    }
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

// The same, each lane holding its share of both parts of every diagonal sum.
template <int GC>
__device__ __forceinline__ void lp_finish_ri(double pre, double pim, const double *dre, const double *dim, int lane,
                                             int w, int W, int g0w, int G, int spin, int stride, int part,
                                             double2 *ekpart, double2 *vbpart) {
  pre = wave_sum_dpp(pre);
  pim = wave_sum_dpp(pim);
  if (lane == 63 && w < W && g0w < G)
    ekpart[((size_t)w * 2 + spin) * stride + part] = make_double2(-0.5 * pre, -0.5 * pim);
  if (vbpart) {
#pragma unroll
    for (int gl = 0; gl < GC; ++gl) {
      const double sre = wave_sum_dpp(dre[gl]), sim = wave_sum_dpp(dim[gl]);
      const int g = g0w + gl;
      if (lane == 63 && w < W && g < G) vbpart[((size_t)spin * W + w) * G + g] = make_double2(sre, sim);
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
// NT = 3 or 2: split-BF16 terms of Ltilde and Theta; NT = 1: the trial split,
// one E term of Ltilde and of Q, with T0 transposed [G4][NR][NR], the inverse scales of
// the Cholesky vectors lsc [G4] and of the walkers qsc [W].
// Contraction runs per stage of the one-product form: one, so that a stage is
// 20 KB and, with the one-plane trace epilogue (28 KB), a workgroup needs 40 KB
// of LDS and three fit on a CU (two 32-deep runs per stage at two workgroups
// per CU measured 9 % slower)
constexpr int kSplitKsub = 1;
// workgroups per CU the one-product kernels are compiled for (registers)
constexpr int kLp16Occupancy1 = 3;
// LDS stages of the 16-bit forms (two; deeper ones, at fewer workgroups per CU,
// measured slower)
__host__ __device__ constexpr int lp16_stages(int) { return 2; }
// Staged planes per stage: the NT terms of the split-BF16 forms, or, for the
// one-product form, KSUB consecutive runs of LKC contraction indices (a stage
// then covers KSUB LKC indices: fewer barriers per contraction)
__host__ __device__ constexpr int lp16_planes(int nt) { return nt == 1 ? kSplitKsub : nt; }
__host__ __device__ constexpr int lp16_kchunk(int nt) { return nt == 1 ? kSplitKsub * LKC : LKC; }
// contraction length of the staged operands: M rounded up to whole chunks
__host__ __device__ constexpr int lp16_kp(int nt, int M) { return (M + lp16_kchunk(nt) - 1) / lp16_kchunk(nt) * lp16_kchunk(nt); }


template <int NR, int NT, typename E = __bf16>
__global__ __launch_bounds__(kThreads, NT == 1 ? kLp16Occupancy1 : NT <= 2 ? 2 : 1) void k_exchange_bf16(const E *__restrict__ LtB,
                                                             const E *__restrict__ ThB, int Kp, int N, int G,
                                                             int W, int stride, int spin,
                                                             double2 *__restrict__ ekpart,
                                                             double2 *__restrict__ vbpart, int ngb, int nwb,
                                                             int group, const float *__restrict__ T0,
                                                             const float *__restrict__ lsc,
                                                             const float *__restrict__ qsc) {
  typedef typename Vec8<E>::type v8;
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
  constexpr int NP = lp16_planes(NT), KCH = lp16_kchunk(NT);
  constexpr int ASZ = NP * ROWS * RS, BSZ = NP * COLS * RS;   // 16-bit elements per stage
  constexpr int AV = NP * ROWS * (LKC / 8), BV = NP * COLS * (LKC / 8);  // 16-byte vectors per stage
  constexpr int TSF = CP + 2;
  static_assert(ROWW % 16 == 0 && CP % 16 == 0 && LKC == 32, "row bases keep the swizzle of the lane's row");
  // Two staging buffers (one barrier per chunk).  The two-term form fits two
  // workgroups per CU (80 KB of LDS, registers for two waves per SIMD), the
  // one-product form three (40 KB, three waves per SIMD); both do the trace
  // epilogue one Cholesky vector of each wave at a time.
  constexpr int NBUF = lp16_stages(NT);
  auto swz = [](int r) { return ((r >> 1) ^ (r >> 2)) & 3; };
  extern __shared__ __attribute__((aligned(16))) unsigned char bsm_raw[];
  E *bsm = reinterpret_cast<E *>(bsm_raw);
  E *sA = bsm, *sB = bsm + NBUF * ASZ;
  // With LDS DMA (global_load_lds_dwordx4: lane L's 16 bytes land at the wave's
  // LDS base + 16 L) a stage is filled straight from memory, 1 KB (16 staged
  // rows) per wave instruction (sources below).
  static_assert(AV % 64 == 0 && BV % 64 == 0, "whole 1 KB blocks");

  int gb, wb;
  tile_of(blockIdx.x, ngb * nwb, ngb, nwb, group, gb, wb);
  const int tid = threadIdx.x, lane = tid & 63;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);   // wave-uniform: LDS stage addresses stay scalar
  const int wy = wv / LWX, wx = wv - (wv / LWX) * LWX;
  const int g0 = gb * LWY * GC, w0 = wb * LWX;
  // plane offsets: the next term, or (one-product form) the next LKC contraction indices
  const size_t aplane = NT == 1 ? (size_t)LKC : (size_t)lp_padded_g(G) * NR * Kp;
  const size_t bplane = NT == 1 ? (size_t)LKC : (size_t)W * CP * Kp;

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
    E *a = sA + buf * ASZ;
    E *b = sB + buf * BSZ;
    const E *la = LtB + q0, *tb = ThB + q0;
#pragma unroll
    for (int r = 0; r < NIA; ++r) {
      const int blk = wv + 4 * r;
      if ((AV / 64) % 4 != 0 && blk >= AV / 64) break;       // uniform in the wave
      const E *src = la + offa[r];
      // non-dependent pointer types: the host pass drops a template kernel whose
      // LDS-DMA builtin takes template-typed pointers
      __builtin_amdgcn_global_load_lds((void *)src, (__attribute__((address_space(3))) void *)((void *)(a + blk * 512)),
                                       16, 0, 0);
    }
#pragma unroll
    for (int r = 0; r < NIB; ++r) {
      const int blk = wv + 4 * r;
      if ((BV / 64) % 4 != 0 && blk >= BV / 64) break;       // uniform in the wave
      const E *src = tb + offb[r];
      __builtin_amdgcn_global_load_lds((void *)src, (__attribute__((address_space(3))) void *)((void *)(b + blk * 512)),
                                       16, 0, 0);
    }
  };

  f4v acc[RT][CT];
#pragma unroll
  for (int i = 0; i < RT; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = f4v{0.f, 0.f, 0.f, 0.f};

  const int nchunk = Kp / KCH;
  // LDS copies per chunk of the wave that issues fewest (the partial vmcnt
  // waits below count in these; a wave that issues more waits a little longer)
  constexpr int CMIN = (AV / 64) / 4 + (BV / 64) / 4;
  // chunks 0 .. NBUF-2 in flight, then wait for chunk 0
  for (int c = 0; c < NBUF - 1; ++c)
    if (c < nchunk) issue(c * KCH, c);
  const int lr = lane & 15, lk = lane >> 4;
  // One-product form: T = T0 + f P with f = (scale of the Cholesky vector) x
  // (scale of the walker), a power of two, so the accumulators start at T0 / f
  // (exact) and end as T / f.  T0 is stored transposed, T0t[g][j][i], so the
  // real part of the lane's four rows i0..i0+3 at column j is one 16-byte load;
  // these loads run while the first stages are copied.
  float tsc[RT];   // f of each row block
  if constexpr (NT == 1) {
    const int g0w = g0 + wy * GC;
    const float qs = qsc[min(w0 + wx, W - 1)];
    const float re = (lr & 1) ? 0.f : 1.f;   // odd lanes hold imaginary parts: T0 adds nothing
#pragma unroll
    for (int rt = 0; rt < RT; ++rt) {
      const int row0 = rt * 16 + 4 * lk;
      const int gl = row0 / NR, i0 = row0 - gl * NR;
      tsc[rt] = lsc[g0w + gl] * qs;
      const float m = re / tsc[rt];
      const float *t0 = T0 + (size_t)(g0w + gl) * NR * NR + i0;
#pragma unroll
      for (int ct = 0; ct < CT; ++ct) {
        const int j = (ct * 16 + lr) >> 1;
        const f4v t = *reinterpret_cast<const f4v *>(t0 + j * NR);
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rt][ct][r] = t[r] * m;
      }
    }
  }
  if (NBUF > 2 && nchunk >= NBUF - 1) AFQMC_WAIT_VMCNT((NBUF - 2) * CMIN);
  else __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  for (int ch = 0; ch < nchunk; ++ch) {
    const int buf = ch % NBUF;
    // into the buffer read in chunk ch - 1 (every wave has passed the barrier after it)
    if (ch + NBUF - 1 < nchunk) issue((ch + NBUF - 1) * KCH, (ch + NBUF - 1) % NBUF);
    const E *a = sA + buf * ASZ + (wy * ROWW + lr) * RS + 8 * (lk ^ swz(lr));
    const E *b = sB + buf * BSZ + (wx * CP + lr) * RS + 8 * (lk ^ swz(lr));
    if constexpr (NT == 1) {
#pragma unroll
      for (int sub = 0; sub < NP; ++sub) {
        v8 ah[RT], bh[CT];
#pragma unroll
        for (int i = 0; i < (RT > CT ? RT : CT); ++i) {
          if (i < RT) ah[i] = *reinterpret_cast<const v8 *>(a + (sub * ROWS + i * 16) * RS);
          if (i < CT) bh[i] = *reinterpret_cast<const v8 *>(b + (sub * COLS + i * 16) * RS);
        }
#pragma unroll
        for (int i = 0; i < RT; ++i)
#pragma unroll
          for (int j = 0; j < CT; ++j) acc[i][j] = mfma16x16x32(ah[i], bh[j], acc[i][j]);
      }
      __builtin_amdgcn_sched_barrier(0);
      // this wave's copies of chunk ch + 1 have landed (later chunks' may not)
      if (NBUF > 2 && ch + NBUF - 1 < nchunk) AFQMC_WAIT_VMCNT((NBUF - 2) * CMIN);
      else __builtin_amdgcn_s_waitcnt(0);
      __syncthreads();
      continue;
    }
    v8 ah[RT], am[RT], bh[CT], bm[CT];
    // the fragments of the first sweep (am x bh) are read first; the other
    // RT + CT reads are spread over that sweep's MFMAs (the group barriers
    // below), so an MFMA waits only on the reads it uses
#pragma unroll
    for (int i = 0; i < (RT > CT ? RT : CT); ++i) {
      if (i < RT) am[i] = *reinterpret_cast<const v8 *>(a + (1 * ROWS + i * 16) * RS);
      if (i < CT) bh[i] = *reinterpret_cast<const v8 *>(b + (0 * COLS + i * 16) * RS);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int j = 0; j < CT; ++j) bm[j] = *reinterpret_cast<const v8 *>(b + (1 * COLS + j * 16) * RS);
#pragma unroll
    for (int i = 0; i < RT; ++i) ah[i] = *reinterpret_cast<const v8 *>(a + (0 * ROWS + i * 16) * RS);
    // one sweep over all accumulators per term, so dependent MFMAs are far
    // apart; the smallest terms first
#define AFQMC_SWEEP(X, Y)                                                                         \
  _Pragma("unroll") for (int i = 0; i < RT; ++i) _Pragma("unroll") for (int j = 0; j < CT; ++j) \
      acc[i][j] = mfma16x16x32(X[i], Y[j], acc[i][j]);
    if constexpr (NT == 3) {
      v8 al[RT], bl[CT];
#pragma unroll
      for (int i = 0; i < RT; ++i) al[i] = *reinterpret_cast<const v8 *>(a + (2 * ROWS + i * 16) * RS);
#pragma unroll
      for (int j = 0; j < CT; ++j) bl[j] = *reinterpret_cast<const v8 *>(b + (2 * COLS + j * 16) * RS);
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
    __builtin_amdgcn_s_waitcnt(0);  // this wave's copies into the other buffer have landed
    __syncthreads();
  }

  if constexpr (NT == 1) {   // T = f (T0 / f + P)
#pragma unroll
    for (int rt = 0; rt < RT; ++rt)
#pragma unroll
      for (int ct = 0; ct < CT; ++ct)
#pragma unroll
        for (int r = 0; r < 4; ++r) acc[rt][ct][r] *= tsc[rt];
  }
  // each lane's partial traces (at most ROWW CP / 64 products) in FP32, the
  // sums over lanes and Cholesky vectors in FP64
  float pre = 0.f, pim = 0.f, dg[2] = {0.f, 0.f};
  if constexpr (NT == 1) {
    // one Cholesky vector of the wave at a time, one plane of S per wave in
    // LDS (the empty asm statements keep the compiler from moving LDS accesses
    // across the phases; the wave's LDS accesses run in order)
    // The diagonal T_ii is read back from the plane by lane i (i < NR) once
    // the plane is in LDS, rather than picked out of the accumulators.
    float *sS = reinterpret_cast<float *>(bsm) + (size_t)wv * lp_s_plane<NR>();
    const bool odd = lr & 1;
    const float *sdiag = sS + min(lane, NR - 1) * (NR + 5);   // S[i][i], row stride NR + 4
    double dre[GC], dim[GC];
#pragma unroll
    for (int pass = 0; pass < GC; ++pass) {
      float a0 = 0.f, a1 = 0.f;   // sum v Re T_ji, sum v Im T_ji
      lp_store_s1<NR, CT, RT>(acc, sS, lane, pass, 0);
      asm volatile("" ::: "memory");
      lp_trace_s1<NR, CT, RT>(acc, sS, lane, a0, pass);
      const float xre = *sdiag;
      asm volatile("" ::: "memory");
      lp_store_s1<NR, CT, RT>(acc, sS, lane, pass, 1);
      asm volatile("" ::: "memory");
      lp_trace_s1<NR, CT, RT>(acc, sS, lane, a1, pass);
      const float xim = *sdiag;
      asm volatile("" ::: "memory");
      pre += odd ? -a1 : a0;
      pim += odd ? a0 : a1;
      dre[pass] = lane < NR ? (double)xre : 0.0;
      dim[pass] = lane < NR ? (double)xim : 0.0;
    }
    lp_finish_ri<GC>((double)pre, (double)pim, dre, dim, lane, w0 + wx, W, g0 + wy * GC, G, spin, stride,
                     gb * LWY + wy, ekpart, vbpart);
    return;
  } else if constexpr (NT == 2) {
    // one Cholesky vector of the wave at a time: S (two planes) per wave in
    // LDS, its diagonal read back by lane i (i < NR).  Lanes read entries
    // other lanes stored: the empty asm statements keep the compiler from
    // moving LDS accesses across the phases or reusing a value loaded in the
    // previous pass (the wave's LDS accesses run in order).
    float *sS = reinterpret_cast<float *>(bsm) + (size_t)wv * 2 * lp_s_plane<NR>();
    const float *sdiag = sS + min(lane, NR - 1) * (NR + 5);   // S[i][i], row stride NR + 4
    double dre[GC], dim[GC];
#pragma unroll
    for (int pass = 0; pass < GC; ++pass) {
      lp_store_s<NR, CT, RT>(acc, sS, lane, pass);
      asm volatile("" ::: "memory");
      lp_trace_s<NR, CT, RT>(acc, sS, lane, pre, pim, pass);
      const float xre = sdiag[0], xim = sdiag[lp_s_plane<NR>()];
      asm volatile("" ::: "memory");
      dre[pass] = lane < NR ? (double)xre : 0.0;
      dim[pass] = lane < NR ? (double)xim : 0.0;
    }
    lp_finish_ri<GC>((double)pre, (double)pim, dre, dim, lane, w0 + wx, W, g0 + wy * GC, G, spin, stride,
                     gb * LWY + wy, ekpart, vbpart);
    return;
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

// ---- trial-split operands ------------------------------------------------------
// power of two that brings a maximum modulus into [2^13, 2^14) (1 for 0 or a
// non-finite maximum): well inside the FP16 and BF16 ranges, exact to undo
__device__ __forceinline__ float pow2_scale(float mx) {
  if (!(mx > 0.f) || !isfinite(mx)) return 1.f;
  int e;
  (void)frexpf(mx, &e);  // mx = m 2^e, m in [0.5, 1)
  return ldexpf(1.f, 14 - e);
}

__device__ __forceinline__ float block_max(float v, float *red) {
  for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) red[wv] = v;
  __syncthreads();
  float m = red[0];
  for (int k = 1; k < (int)(blockDim.x >> 6); ++k) m = fmaxf(m, red[k]);
  __syncthreads();
  return m;
}

// One workgroup per Cholesky vector g < G4 (the padded count): the scaled
// 16-bit plane LtB[g][i][q] (q < Kp, zero for q >= M, i >= N or g >= G), its
// inverse scale lsc[g], and T0 transposed, T0t[g][j][i] = sum_q Ltilde[i][q]
// Psi[q][off + j] (zero outside i, j < N), from LtS[g][q][i] (FP64, rows padded
// to NR).
template <typename E>
__global__ __launch_bounds__(kThreads) void k_lt_split(const double *__restrict__ LtS, const double *__restrict__ trial,
                                                      int G, int M, int Nt, int off, int N, int NR, int Kp,
                                                      E *__restrict__ LtB, float *__restrict__ T0,
                                                      float *__restrict__ lsc) {
  __shared__ float red[kThreads / 64];
  const int g = blockIdx.x, tid = threadIdx.x;
  const double *L = LtS + (size_t)g * M * NR;
  float mx = 0.f;
  if (g < G)
    for (int e = tid; e < M * NR; e += blockDim.x) mx = fmaxf(mx, fabsf((float)L[e]));
  const float sc = pow2_scale(block_max(mx, red));
  if (tid == 0) lsc[g] = 1.f / sc;
  for (int e = tid; e < NR * Kp; e += blockDim.x) {
    const int i = e / Kp, q = e - (e / Kp) * Kp;
    const double x = (g < G && q < M && i < N) ? L[(size_t)q * NR + i] : 0.0;
    LtB[(size_t)g * NR * Kp + e] = (E)(float)(x * (double)sc);
  }
  for (int e = tid; e < NR * NR; e += blockDim.x) {
    const int j = e / NR, i = e - (e / NR) * NR;      // stored transposed: T0t[g][j][i]
    double a = 0.0;
    if (g < G && i < N && j < N)
      for (int q = 0; q < M; ++q) a = fma(L[(size_t)q * NR + i], trial[(size_t)q * Nt + off + j], a);
    T0[(size_t)g * NR * NR + e] = (float)a;
  }
}

// Q = Theta - Psi of one spin block (re/im interleaved over CP = 2 NR columns,
// zero past 2N), scaled by a power of two per walker and written K-contiguous,
// ThB[w][c][q] (q < Kp, zero for q >= M).  First one workgroup per walker finds
// max |Q| and stores the inverse scale in qsc[w] (sixteen waves, so that one
// workgroup per CU keeps enough loads in flight; a maximum does not depend on
// the order); then one workgroup per (32 rows q, walker) transposes its rows
// through LDS.
constexpr int kQmaxThreads = 1024;
__global__ __launch_bounds__(kQmaxThreads) void k_q_max(const double2 *__restrict__ theta,
                                                       const double *__restrict__ trial, int M, int Nt, int off,
                                                       int N, float *__restrict__ qsc) {
  __shared__ float red[kQmaxThreads / 64];
  const int w = blockIdx.x, tid = threadIdx.x;
  const double2 *th = theta + (size_t)w * M * Nt + off;
  float mx = 0.f;
  for (int e = tid; e < M * N; e += blockDim.x) {
    const int q = e / N, j = e - (e / N) * N;
    const double2 z = th[(size_t)q * Nt + j];
    mx = fmaxf(mx, fmaxf(fabsf((float)(z.x - trial[(size_t)q * Nt + off + j])), fabsf((float)z.y)));
  }
  const float sc = pow2_scale(block_max(mx, red));
  if (tid == 0) qsc[w] = 1.f / sc;
}

template <typename E>
__global__ __launch_bounds__(kThreads) void k_q_split(const double2 *__restrict__ theta,
                                                     const double *__restrict__ trial, int M, int Nt, int off, int N,
                                                     int CP, int Kp, const float *__restrict__ qsc,
                                                     E *__restrict__ ThB) {
  extern __shared__ float qsm[];  // [32][CP + 1]
  const int w = blockIdx.y, q0 = blockIdx.x * 32, tid = threadIdx.x;
  const double2 *th = theta + (size_t)w * M * Nt + off;
  const double sc = 1.0 / (double)qsc[w];   // a power of two
  for (int e = tid; e < 32 * CP; e += blockDim.x) {
    const int qq = e / CP, c = e - (e / CP) * CP;
    const int q = q0 + qq;
    double v = 0.0;
    if (q < M && c < 2 * N) {
      const double2 z = th[(size_t)q * Nt + (c >> 1)];
      v = (c & 1) ? z.y : z.x - trial[(size_t)q * Nt + off + (c >> 1)];
    }
    qsm[qq * (CP + 1) + c] = (float)(v * sc);
  }
  __syncthreads();
  for (int e = tid; e < 32 * CP; e += blockDim.x) {
    const int c = e / 32, qq = e - (e / 32) * 32;
    ThB[((size_t)w * CP + c) * Kp + q0 + qq] = (E)qsm[qq * (CP + 1) + c];
  }
}

// ---- dispatch -------------------------------------------------------------------
namespace {
using F32Kernel = void (*)(const float *, const float *, int, int, int, int, int, int, double2 *, double2 *, int,
                           int, int);
using BFKernel = void (*)(const __bf16 *, const __bf16 *, int, int, int, int, int, int, double2 *, double2 *, int,
                          int, int, const float *, const float *, const float *);
using HKernel = void (*)(const _Float16 *, const _Float16 *, int, int, int, int, int, int, double2 *, double2 *, int,
                         int, int, const float *, const float *, const float *);

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
HKernel pick_h1(int nr) {
  switch (nr) {
    case 8: return k_exchange_bf16<8, 1, _Float16>;
    case 16: return k_exchange_bf16<16, 1, _Float16>;
    case 24: return k_exchange_bf16<24, 1, _Float16>;
    case 32: return k_exchange_bf16<32, 1, _Float16>;
    case 40: return k_exchange_bf16<40, 1, _Float16>;
    case 48: return k_exchange_bf16<48, 1, _Float16>;
    default: return nullptr;
  }
}
// 16-bit terms per operand of a 16-bit precision (0: not one): the split-BF16
// forms, or one term of the trial split
int bf_terms(int precision) {
  return precision == AFQMC_BF16X3_CONTRACT ? 3
         : precision == AFQMC_BF16X2_CONTRACT ? 2
         : (precision == AFQMC_FP16_TSPLIT_CONTRACT || precision == AFQMC_BF16_TSPLIT_CONTRACT) ? 1
                                                                                                : 0;
}
bool tsplit(int precision) { return bf_terms(precision) == 1; }
bool f16(int precision) { return precision == AFQMC_FP16_TSPLIT_CONTRACT; }
BFKernel pick_bf(int nr, int nt) {
  return nt == 3 ? pick_bf_nt<3>(nr) : nt == 2 ? pick_bf_nt<2>(nr) : nt == 1 ? pick_bf_nt<1>(nr) : nullptr;
}
const void *pick_lp16(int precision, int nr) {
  return f16(precision) ? reinterpret_cast<const void *>(pick_h1(nr))
                        : reinterpret_cast<const void *>(pick_bf(nr, bf_terms(precision)));
}
size_t pad256(size_t b) { return (b + 255) / 256 * 256; }
// byte layout of the trial-split operands: lhs = plane | T0 | lsc, rhs = plane | qsc
struct SplitLayout {
  size_t lplane, t0, lsc, lhs, rplane, qsc, rhs;
};
SplitLayout split_layout(int G, int M, int W, int nr) {
  const size_t kp = lp16_kp(1, M), g4 = lp_padded_g(G), cp = 2 * (size_t)nr;
  SplitLayout l;
  l.lplane = 0;
  l.t0 = pad256(g4 * nr * kp * 2);
  l.lsc = l.t0 + pad256(g4 * nr * nr * sizeof(float));
  l.lhs = l.lsc + pad256(g4 * sizeof(float));
  l.rplane = 0;
  l.qsc = pad256((size_t)W * cp * kp * 2);
  l.rhs = l.qsc + pad256((size_t)W * sizeof(float));
  return l;
}
size_t lds_f32(int nr) {
  const int gc = (nr % 16 == 0) ? 1 : 2, roww = gc * nr, cp = 2 * nr;
  const size_t stage = 2ull * (LKC * LWY * roww + LWX * LKC * cp) * sizeof(float);
  const size_t epi = 4ull * roww * (cp + 2) * sizeof(float);
  return stage > epi ? stage : epi;
}
size_t lds_bf(int nr, int nt) {
  const int gc = (nr % 16 == 0) ? 1 : 2, roww = gc * nr, cp = 2 * nr;
  const size_t nbuf = lp16_stages(nt);
  const size_t stage = nbuf * lp16_planes(nt) * (LWY * roww + LWX * cp) * LKC * sizeof(__bf16);
  const size_t epi = nt == 1 ? 4ull * (nr * (nr + 4) + 8) * sizeof(float)
                     : nt == 2 ? 4ull * 2 * (nr * (nr + 4) + 8) * sizeof(float) : 4ull * roww * (cp + 2) * sizeof(float);
  return stage > epi ? stage : epi;
}
}  // namespace

bool lp_exchange_supported(int precision, int nr) {
  if (precision == AFQMC_FP32_CONTRACT) return pick_f32(nr) && lds_f32(nr) <= 160 * 1024;
  const int nt = bf_terms(precision);
  if (nt) return pick_lp16(precision, nr) && lds_bf(nr, nt) <= 160 * 1024;
  return false;
}

size_t lp_operand_elems(int precision, int G, int M, int W, int nr, bool lhs) {
  const int kp = lp16_kp(bf_terms(precision), M);
  if (precision == AFQMC_FP32_CONTRACT) return lhs ? (size_t)G * M * nr : (size_t)W * M * 2 * nr;
  const size_t nt = bf_terms(precision);
  return lhs ? nt * lp_padded_g(G) * nr * kp : nt * W * 2 * nr * kp;
}

size_t lp_operand_bytes(int precision, int G, int M, int W, int nr, bool lhs) {
  if (tsplit(precision)) {
    const SplitLayout l = split_layout(G, M, W, nr);
    return lhs ? l.lhs : l.rhs;
  }
  const size_t esz = precision == AFQMC_FP32_CONTRACT ? 4 : 2;
  return esz * lp_operand_elems(precision, G, M, W, nr, lhs);
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
  } else if (tsplit(s.precision)) {
    const int kp = lp16_kp(bf_terms(s.precision), s.M);
    const SplitLayout l = split_layout(s.G, s.M, s.W, p.NR);
    unsigned char *base = static_cast<unsigned char *>(s.lp_lhs[spin]);
    float *T0 = reinterpret_cast<float *>(base + l.t0), *lsc = reinterpret_cast<float *>(base + l.lsc);
    const int off = spin ? s.Na : 0;
    if (f16(s.precision))
      hipLaunchKernelGGL(k_lt_split<_Float16>, dim3(lp_padded_g(s.G)), dim3(kThreads), 0, st, s.LtS[spin], s.trial,
                         s.G, s.M, s.Nt, off, p.N, p.NR, kp, reinterpret_cast<_Float16 *>(base), T0, lsc);
    else
      hipLaunchKernelGGL(k_lt_split<__bf16>, dim3(lp_padded_g(s.G)), dim3(kThreads), 0, st, s.LtS[spin], s.trial,
                         s.G, s.M, s.Nt, off, p.N, p.NR, kp, reinterpret_cast<__bf16 *>(base), T0, lsc);
  } else {
    const int kp = lp16_kp(bf_terms(s.precision), s.M);
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
      e = hipFuncSetAttribute(pick_lp16(s.precision, p.NR), hipFuncAttributeMaxDynamicSharedMemorySize,
                              (int)lds_bf(p.NR, bf_terms(s.precision)));
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
  } else if (tsplit(s.precision)) {
    const int kp = lp16_kp(bf_terms(s.precision), s.M);
    const SplitLayout l = split_layout(s.G, s.M, s.W, p.NR);
    unsigned char *base = static_cast<unsigned char *>(s.lp_rhs[spin]);
    float *qsc = reinterpret_cast<float *>(base + l.qsc);
    const size_t lds = 32ull * (CP + 1) * sizeof(float);
    hipLaunchKernelGGL(k_q_max, dim3(W), dim3(kQmaxThreads), 0, st, theta, s.trial, s.M, s.Nt, off, p.N, qsc);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (f16(s.precision))
      hipLaunchKernelGGL(k_q_split<_Float16>, dim3(kp / 32, W), dim3(kThreads), lds, st, theta, s.trial, s.M, s.Nt,
                         off, p.N, CP, kp, qsc, reinterpret_cast<_Float16 *>(base));
    else
      hipLaunchKernelGGL(k_q_split<__bf16>, dim3(kp / 32, W), dim3(kThreads), lds, st, theta, s.trial, s.M, s.Nt,
                         off, p.N, CP, kp, qsc, reinterpret_cast<__bf16 *>(base));
  } else {
    const int kp = lp16_kp(bf_terms(s.precision), s.M);
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
    const int kp = lp16_kp(bf_terms(s.precision), s.M);
    const int nt = bf_terms(s.precision);
    const float *T0 = nullptr, *lsc = nullptr, *qsc = nullptr;
    if (tsplit(s.precision)) {
      const SplitLayout l = split_layout(s.G, s.M, s.W, p.NR);
      const unsigned char *lb = static_cast<const unsigned char *>(s.lp_lhs[spin]);
      const unsigned char *rb = static_cast<const unsigned char *>(s.lp_rhs[spin]);
      T0 = reinterpret_cast<const float *>(lb + l.t0);
      lsc = reinterpret_cast<const float *>(lb + l.lsc);
      qsc = reinterpret_cast<const float *>(rb + l.qsc);
    }
    if (f16(s.precision))
      hipLaunchKernelGGL(pick_h1(p.NR), grid, dim3(kThreads), lds_bf(p.NR, nt), st,
                         static_cast<const _Float16 *>(s.lp_lhs[spin]), static_cast<const _Float16 *>(s.lp_rhs[spin]),
                         kp, p.N, s.G, W, s.ex_stride, spin, s.ekpart, vbpart, ngb, nwb, s.ex_group, T0, lsc, qsc);
    else
      hipLaunchKernelGGL(pick_bf(p.NR, nt), grid, dim3(kThreads), lds_bf(p.NR, nt), st,
                         static_cast<const __bf16 *>(s.lp_lhs[spin]), static_cast<const __bf16 *>(s.lp_rhs[spin]), kp,
                         p.N, s.G, W, s.ex_stride, spin, s.ekpart, vbpart, ngb, nwb, s.ex_group, T0, lsc, qsc);
  }
  return hipGetLastError();
}

}  // namespace afqmc
