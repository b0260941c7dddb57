// Internal declarations of libafqmc: per-system device state and kernel launchers.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "afqmc.h"

namespace afqmc {

constexpr int kMaxSpinOrbitals = 56;  // widest spin block: N^2 complex fits the 64 KiB LDS budget
constexpr int kThreads = 256;
// learned control variate: network sizes and the largest walker count of its subset draw
constexpr int kCvFeatures = 10, kCvHidden = 128;
constexpr int kCvParams = kCvHidden * kCvFeatures + kCvHidden + kCvHidden * kCvHidden + kCvHidden + 2 * kCvHidden + 2;
constexpr int kCvNorm = 2 * kCvFeatures + 4;
constexpr int kCvMaxWalkers = 4096;
constexpr int kCvGradBlock = 16;  // samples per workgroup of the network's gradient kernel

// Device buffers and scalars of one system.  Layouts (row-major):
//   L      [G][M][M]     Cholesky vectors
//   LtT    [G][M][Nt]    half-rotated vectors, LtT[g][q][i'] = (Psi_s^T L^g)_{i q}
//   htT    [M][Nt]       htT[q][i'] = (Psi_s^T h)_{i q}
//   trial  [M][Nt]
//   B1     [M][M]        exp(-dt/2 H1)
//   lmf    [G]           mean-field shift l_g (m_g = i l_g)
// Workspaces sized for W walkers:
//   theta  [W][M][Nt] double2        Green's-function factor Theta
//   fbpart [ks][W][G] double2        split-K partial sums of vbias
//   yp     [W][2][G]                 sqrt(dt) * (Im y, -Re y): rows of the VHS product
//   vhs    [W][2][M][M]              A = sqrt(dt) V_HS as real and imaginary planes
//   tA,tB,tacc [W][M][Nt] double2    Taylor-series term ping-pong and accumulator
//   logo_now, logo_new [W] double2   log overlaps before/after the step
//   stat_now, stat_new [W] uint32    singular markers of the two LU passes
//   wsc    [W][6]                    sum x.xbar, sum xbar.xbar, sum y.l (complex)
//   e1, ej [W] double2; ekpart [W][2][ngb] double2
// Launch plan of the MFMA exchange kernel for one spin block of width N.
struct ExchangePlan {
  int N = 0, NR = 0, GC = 1, RT = 0, CT = 0, WX = 4, WY = 1;
  int ngroups = 0;  // partial sums written per (walker, spin)
  int nwg = 0;      // workgroups along the Cholesky index
  size_t lds = 0;
  bool mfma = false;
};
ExchangePlan exchange_plan(int N, int G, int wx);

struct System {
  int M = 0, Na = 0, Nb = 0, Nt = 0, G = 0, W = 0;
  double dt = 0, sqdt = 0, ecore = 0, e_hf = 0, e_shift = 0, const_c = 0;
  uint64_t bytes = 0;

  double *eshift = nullptr;             // [1] E_T of the weight update, on the device
  double *L = nullptr, *LtT = nullptr, *htT = nullptr, *trial = nullptr, *B1 = nullptr, *lmf = nullptr;
  double *LtS[2] = {nullptr, nullptr};  // per spin [G][M][NR]: half-rotated, rows padded for the exchange
  double *Lp = nullptr;                 // [G][M(M+1)/2] packed upper triangles of the L^g
  double *vhsp = nullptr;               // [W][2][M(M+1)/2] packed V_HS planes
  float *Lp32 = nullptr;                // FP32 propagation: packed L^g in FP32, [G][ldlp32]
  long ldlp32 = 0;                      // M(M+1)/2 rounded up to a multiple of 4
  // FP32 propagation: V_HS planes and Taylor terms in single precision
  bool prop32 = false;
  float *vhs32 = nullptr;                // [W][2][M][M]
  float2 *tA32 = nullptr, *tB32 = nullptr;  // [W][M][Nt]
  double2 *theta = nullptr, *fbpart = nullptr, *tA = nullptr, *tB = nullptr, *tacc = nullptr;
  double *yp = nullptr, *vhs = nullptr, *wsc = nullptr;
  double2 *logo_now = nullptr, *logo_new = nullptr, *e1 = nullptr, *ej = nullptr, *ekpart = nullptr;
  uint32_t *stat_now = nullptr, *stat_new = nullptr;
  double2 *opart = nullptr;    // per-spin-block scratch of the overlap and Gram-Schmidt kernels, [W][2]
  uint32_t *ospart = nullptr;   // [W][2]
  // second stream of the Taylor terms (the walkers' second half), forked from
  // and joined into the system's stream, so that one half's launch tail
  // overlaps the other half's work
  hipStream_t half_stream = nullptr;
  hipEvent_t half_fork = nullptr, half_join = nullptr;

  int fb_ksplit = 1;  // split-K slices of the force-bias contraction
  int ex_gb = 1;      // Cholesky vectors per workgroup of the VALU exchange kernel
  int ex_ngb = 1;     // its number of workgroups along G
  size_t ex_lds = 0;  // its dynamic LDS
  bool use_mfma_gemm = true;   // MFMA kernels for force bias, V_HS, B1 and Taylor terms
  bool taylor_kernel = true;   // the dedicated Taylor-term kernel (else the generic MFMA GEMM)
  int vhs_shape = 0;           // tile shape of the V_HS GEMM (kVhsShapes candidates)
  int taylor_shape = 0;        // tile shape of the Taylor-term kernel (taylor_shapes(s) candidates)
  bool pack_chol = true;       // V_HS from the packed upper triangles of the L^g
  bool free_full = false;      // free projection through both V_HS planes (comparison runs)
  bool ex_mfma = false;        // MFMA exchange kernel in use (both spin blocks)
  ExchangePlan ex_plan[2];     // its per-spin plans
  int ex_group = 0;            // tile order of the MFMA exchange launches (see tile_of)
  // learned control variate of the exchange energy
  int ex_mode = AFQMC_EX_FULL;
  int cv_k = 0;                          // walkers with exact exchange per call
  uint64_t cv_seed = 7;
  float *cv_params = nullptr, *cv_m = nullptr, *cv_v = nullptr;  // [kCvParams] each
  double *cv_norm = nullptr;             // [kCvNorm]
  double *cv_feat = nullptr;             // [W][kCvFeatures]
  double *KtT = nullptr;                 // [M][Nt]: KtT[q][i'] = K_s[i][q], K_s = sum_g (Ltilde Psi_s) Ltilde
  double2 *cv_lin = nullptr;             // [W] sum_s Tr(K_s Theta_s) (the first-order exchange feature)
  double2 *cv_f = nullptr;               // [W] predictions
  int *cv_sel = nullptr, *cv_pos = nullptr;  // [W]
  uint64_t *cv_counter = nullptr;        // [2]: next call, last call
  double2 *cv_theta = nullptr;           // [cv_k][M][Nt] Theta of the subset
  int ex_stride = 1;           // partials per (walker, spin) in ekpart
  int ex_nparts[2] = {0, 0};   // partials actually written per spin
  // Theta / vbias partials in `theta` / `fbpart` belong to these walker buffers
  const void *cache_phi = nullptr;
  int fb_slices = 0;           // slices of fbpart holding the current vbias
  // reduced-precision exchange (and force bias): per-spin operands
  int precision = AFQMC_FP64;
  // Ltilde as FP32 [G][M][NR] or 16-bit planes [NT][G4][NR][Kp] (trial split: one plane, then T0 and scales)
  void *lp_lhs[2] = {nullptr, nullptr};
  // Theta as FP32 [W][M][CP] or 16-bit planes [NT][W][CP][Kp] (trial split: Q = Theta - Psi, then scales)
  void *lp_rhs[2] = {nullptr, nullptr};
};

// Reduced-precision exchange (k_exchange_lp.hip).
bool lp_exchange_supported(int precision, int nr);
// the split-BF16 kernels address their operand planes with 32-bit element offsets
bool lp_operands_addressable(int precision, int G, int M, int W, int nr);
size_t lp_operand_elems(int precision, int G, int M, int W, int nr, bool lhs);
size_t lp_operand_bytes(int precision, int G, int M, int W, int nr, bool lhs);
hipError_t lp_prepare_lhs(const System &s, int spin, hipStream_t st);
hipError_t lp_enable_lds(const System &s);
// Reduced-precision copy of one spin block of Theta (the right operand of the
// exchange contraction), then the exchange of that spin block from it.
hipError_t lp_prepare_rhs(const System &s, const double2 *theta, int W, int spin, hipStream_t st);
hipError_t launch_exchange_lp(const System &s, int W, int spin, hipStream_t st, double2 *vbpart);

struct Options {
  int precision = AFQMC_FP64;
  int taylor_order = 6;
  double fb_cap = 1.0;
  int ex_mode = AFQMC_EX_FULL;
  double cv_fraction = 0.125;
  uint64_t cv_seed = 7;
  int prop_precision = AFQMC_FP64;
};

// ---- kernel launchers (each returns the hipGetLastError() of its launch) ----

// Generic strided FP64 GEMM: C(i,j) = alpha * sum_k A(i,k) B(k,j) + beta * C(i,j)
// with A(i,k) = A[b*sab + i*sai + k*sak], B(k,j) = B[b*sbb + k*sbk + j*sbj],
// C(i,j) = C[b*scb + s*scs + i*sci + j*scj] where s is the split-K slice.
struct GemmArgs {
  int m = 0, n = 0, k = 0, batch = 1, ksplit = 1;
  const double *A = nullptr; long sai = 0, sak = 0, sab = 0;
  const double *B = nullptr; long sbk = 0, sbj = 0, sbb = 0;
  double *C = nullptr; long sci = 0, scj = 0, scb = 0, scs = 0;
  double alpha = 1.0, beta = 0.0;
  // MFMA GEMM extras: contraction split point and plane offset of a complex A
  // held as planes, a second output accumulated with the same values, and
  // interleaved-complex output rows.
  int khalf = 0;
  long aplane = 0;
  double *C2 = nullptr;
  int cplx_rows = 0;
};
hipError_t gemm_f64(const GemmArgs &a, hipStream_t st);
hipError_t gemm_vhs_mfma(const GemmArgs &a, hipStream_t st, int shape);
constexpr int kVhsShapes = 4;   // tile shapes of the V_HS GEMM the tuner tries
hipError_t gemm_b1_mfma(const GemmArgs &a, hipStream_t st);
hipError_t gemm_taylor_mfma(const GemmArgs &a, hipStream_t st);
hipError_t gemm_fb_mfma(const GemmArgs &a, hipStream_t st);
hipError_t gemm_nn_mfma(const GemmArgs &a, hipStream_t st);

// Overlap, log-determinant and (optionally) Theta for every walker.
// part: [W][2] double2 and spart: [W][2] uint32 scratch (per spin block)
hipError_t launch_ovlp_theta(const double2 *phi, const double *trial, int M, int Na, int Nb, int W,
                             double2 *theta, double2 *logo, uint32_t *stat, uint32_t *flags_or, hipStream_t st,
                             double2 *part, uint32_t *spart);
hipError_t ovlp_enable_lds(int nmax);
// Modified Gram-Schmidt per spin block, log_ovlp -= sum log R_ii.
// scratch: [W][2] doubles
hipError_t launch_mgs(double2 *phi, int M, int Na, int Nb, int W, double2 *logo, hipStream_t st, double *scratch);

// Force bias: split-K contraction into fbpart, then the epilogues.
hipError_t launch_force_bias_gemm(const System &s, const double2 *theta, int W, hipStream_t st);
// The epilogues sum the `nslices` slices [nslices][W][G] of fbpart (split-K
// partials of the force-bias GEMM, or the two spin parts from the exchange).
hipError_t launch_fb_propagate_epilogue(const System &s, const Options &o, const double *x, int W,
                                        uint32_t *flags, int nslices, hipStream_t st);
hipError_t launch_fb_energy_epilogue(const System &s, int W, double2 *vbias_out, int nslices, hipStream_t st);

// Two-body generator A = sqrt(dt) V_HS for every walker.
// imag_only: form only the imaginary planes (rows (w, 1)); the real planes are
// left as they are and must not be read (a purely imaginary V_HS)
hipError_t launch_vhs(const System &s, int W, hipStream_t st, bool imag_only = false);
// out_w = B1 in_w for every walker (real M x M times complex M x Nt).
hipError_t launch_b1(const System &s, const double2 *in, double2 *out, int W, hipStream_t st);
// Taylor term: tout = alpha * A_w tin; tacc += tout.
// kbeg = M skips the real plane of V_HS (zero for free projection); only the
// MFMA Taylor kernels take kbeg != 0 (free_half_supported)
hipError_t launch_taylor_term(const System &s, const double2 *tin, double2 *tout, double alpha, int W,
                              hipStream_t st, int kbeg = 0);
bool free_half_supported(const System &s);
// Weight update of the phaseless step.
hipError_t launch_weight_update(const System &s, const afqmc_walkers &w, int W, hipStream_t st);

// Energies.
hipError_t launch_energy_e1(const System &s, const double2 *theta, int W, hipStream_t st);
// out[w] = sum_{q,i'} mat[q][i'] theta[w][q][i'] (K = M Nt), complex
hipError_t launch_trace_half(const double *mat, const double2 *theta, int W, long K, double2 *out, hipStream_t st);
// With vbpart (MFMA path only) the kernel also writes this spin's trace of T,
// sum_i T^{g s}_ii, to vbpart[s][w][g]: the spin parts of vbias_g.
// spin = 0 or 1 launches that spin block only, -1 both.
hipError_t launch_exchange(const System &s, const double2 *theta, int W, hipStream_t st,
                           double2 *vbpart = nullptr, int spin = -1);
hipError_t exchange_enable_lds(const System &s);
// LtS[g][q][i] = LtT[g][q][off + i] for i < N, zero for N <= i < NR.
hipError_t launch_pad_half_rotated(const double *LtT, int G, int M, int Nt, int off, int N, int NR, double *LtS,
                                   hipStream_t st);
hipError_t launch_energy_combine(const System &s, int W, double2 *e_out, hipStream_t st);
hipError_t launch_estimator(const double *weight, const double2 *e_out, int W, double *est, hipStream_t st);
// E_T: set to a value, or to the mixed estimate of a block of estimator records [nsteps][4]
hipError_t launch_set_e_shift(const System &s, double e_shift, hipStream_t st);
hipError_t launch_block_e_shift(const System &s, const double *est, int nsteps, hipStream_t st);

// Set-up helpers.
hipError_t launch_row_dot(const double *A, const double *v, long len, int rows, double *out, hipStream_t st);
hipError_t launch_sum_slices(const double *parts, int nslices, long n, double alpha, double *inout,
                             hipStream_t st);
hipError_t launch_add_identity(double *A, int M, double diag, hipStream_t st);
hipError_t launch_axpby(const double *x, double a, double *y, double b, long n, hipStream_t st);
hipError_t launch_zero2(double2 *p, long n, hipStream_t st);
hipError_t launch_fill_pattern2(double2 *p, long n, hipStream_t st);
hipError_t launch_pack_upper(const System &s, hipStream_t st);
// FP32 propagation (k_taylor32.hip)
bool prop32_supported(int M, int Nt);
hipError_t launch_taylor_f32(const System &s, const float2 *tin, float2 *tout, double alpha, int W, hipStream_t st,
                             int kbeg = 0);
hipError_t launch_c128_to_c64(const double2 *in, long n, float2 *out, hipStream_t st);
hipError_t launch_unpack_f32(const System &s, int W, hipStream_t st, bool imag_only = false);
hipError_t launch_pack_to_f32(const double *in, long n, long rows, long ldo, float *out, hipStream_t st);
// V_HS of FP32 propagation from Lp32 (FP32 GEMM), unpacked into the FP32 planes
hipError_t launch_vhs_f32(const System &s, int W, hipStream_t st, bool imag_only);
// comb population control (k_popctl.hip); parents_out may be NULL
// free projection
hipError_t launch_free_fields(const System &s, const double *x, int W, uint32_t *flags, hipStream_t st);
hipError_t launch_free_amplitude(const System &s, const afqmc_walkers &wk, double2 *amp, int W, hipStream_t st);
hipError_t launch_free_estimator(const double *weight, const uint32_t *flags, const double2 *amp, const double2 *e,
                                 int W, double *est, hipStream_t st);
hipError_t launch_comb(const System &s, double *weight, double2 *phi, double2 *logo, uint32_t *flags, const double *u,
                       int *parents_out, hipStream_t st);
// the synthetic Cholesky tensor of the counter recipe (see afqmc_system_desc)
hipError_t launch_gen_chol(const System &s, uint64_t seed, const double *fac, double root3, hipStream_t st);
// dedicated Taylor-term kernel (k_taylor.hip)
bool taylor_mfma_supported(int M, int Nt);
// acc: 1 tacc += tout; 0 tacc untouched (tin may be tacc); 2 tacc += tin + tout
hipError_t launch_taylor_mfma(const System &s, const double2 *tin, double2 *tout, double alpha, int W,
                              hipStream_t st, int kbeg = 0, int w0 = 0, int acc = 1);
// the Taylor terms of walkers [w0, w0 + W) can run as a launch of their own
// (the dedicated three-product kernel)
bool taylor_walker_split(const System &s);
// tile shapes of the dedicated Taylor kernel in use (FP64 or FP32 propagation)
int taylor_shapes(const System &s);

// learned control variate (k_cv.hip)
hipError_t cv_enable_lds();
hipError_t launch_cv_init(const System &s, uint64_t seed, hipStream_t st);
hipError_t launch_cv_zero(void *p, size_t bytes, hipStream_t st);
hipError_t launch_cv_features(const System &s, int W, double *feat, hipStream_t st);
// K_s of the first-order exchange feature, from LtT and the trial (set-up; t0: [G][Nt][Nt] scratch)
hipError_t launch_cv_kmat(System &s, double *t0, hipStream_t st);
hipError_t launch_cv_predict(const System &s, const double *feat, long n, double2 *f, hipStream_t st);
hipError_t launch_cv_subset(const System &s, int W, int k, uint64_t seed, hipStream_t st);
hipError_t launch_cv_gather(const System &s, int k, hipStream_t st);
hipError_t launch_cv_combine(const System &s, int W, int k, double2 *e_out, hipStream_t st);
hipError_t launch_cv_ek(const System &s, int W, double2 *ek, hipStream_t st);
hipError_t launch_cv_stats(const double *feat, const double2 *ek, long n, double *norm, hipStream_t st);
hipError_t launch_cv_standardise(const double *feat, const double2 *ek, long n, const double *norm, float *X,
                                 float *T, hipStream_t st);
int cv_grad_workgroups(long nb);
hipError_t launch_cv_grad(const float *P, const float *X, const float *T, long n0, long nb, float *part,
                          double *lpart, float *grad, double loss_scale, double *loss, hipStream_t st);
hipError_t launch_cv_adam(float *P, const float *grad, float *m, float *v, double lr, long t, hipStream_t st);

// Exchange launch geometry for a spin block width.
void exchange_geometry(int nmax, int *gb, size_t *lds);

}  // namespace afqmc
