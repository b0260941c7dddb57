/*
 * afqmc.h -- C ABI of the MI355X phaseless-AFQMC walker step (libafqmc.so).
 *
 * The library implements one time step of phaseless auxiliary-field quantum
 * Monte Carlo for an ab-initio Hamiltonian whose two-electron integrals are
 * given as Cholesky vectors (arXiv:2406.16238, Sec. 2, eqs. qcham and
 * chol_decomp), with a single Slater-determinant trial (Sec. 3.3, the
 * single-determinant trial object) and unrestricted walkers.  Every step of the
 * path runs in the library's own HIP kernels on the caller's stream.
 *
 * Conventions shared by all calls
 * -------------------------------
 * Sizes: M = nbasis, Na = nalpha, Nb = nbeta, Nt = Na + Nb, G = nchol,
 *        W = nwalkers (fixed per system at set-up).
 * Complex numbers are interleaved (re, im) pairs of doubles ("double2").
 * All matrices are row-major.
 * Walker slab phi: device double2 [W][M][Nt]; columns 0..Na-1 are the alpha
 *   orbitals, Na..Nt-1 the beta orbitals (the trial's hstack([orbs_a, orbs_b])
 *   layout).
 * Ownership: the caller allocates and owns every walker, field and output
 *   buffer; the context owns everything derived from the Hamiltonian and its
 *   own workspaces, and frees them in afqmc_destroy.  No call dereferences a
 *   caller pointer after it returns (afqmc_step and afqmc_run_block compare
 *   walker addresses with the previous call's; see there).
 * Streams: every call except afqmc_setup_hamiltonian enqueues its kernels on
 *   `hip_stream` (a hipStream_t, NULL = the default stream) and returns
 *   without synchronising.  The returned status covers argument validation and
 *   launch errors only; numerical trouble is reported per walker in the flag
 *   word.  Calls that share a context must not overlap in time (they share the
 *   context's workspaces): issue them on one stream, or synchronise.
 * Errors: no call aborts or throws.  On a non-OK status the outputs are
 *   unspecified, the context stays valid, and afqmc_last_error() returns a
 *   message for the calling thread.
 */
#ifndef AFQMC_H
#define AFQMC_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct afqmc_ctx afqmc_ctx;

typedef enum {
  AFQMC_OK = 0,
  AFQMC_ERR_ARG = 1,          /* invalid argument; nothing was launched       */
  AFQMC_ERR_OOM = 2,          /* device memory (or mem_limit_bytes) exhausted */
  AFQMC_ERR_HIP = 3,          /* a HIP runtime call or launch failed          */
  AFQMC_ERR_UNSUPPORTED = 4   /* valid but outside what the library supports */
} afqmc_status;

/* Precision of the force-bias and exchange contractions (overlap LU,
 * determinant ratios, re-orthogonalisation and weights are always FP64):
 * FP32; split BF16 with three or two bfloat16 terms per operand (six or three
 * products); or the trial split, Theta = Psi + Q, T = Ltilde Psi (exact, set
 * up once) + Ltilde Q with Ltilde and Q in one FP16 or BF16 term each (one
 * product, scaled by powers of two per Cholesky vector and per walker).  All
 * accumulate in FP32 on MFMA; spin blocks of at most 48 orbitals. */
enum {
  AFQMC_FP64 = 0,
  AFQMC_FP32_CONTRACT = 1,
  AFQMC_BF16X3_CONTRACT = 2,
  AFQMC_BF16X2_CONTRACT = 3,
  AFQMC_FP16_TSPLIT_CONTRACT = 4,
  AFQMC_BF16_TSPLIT_CONTRACT = 5
};

/* Per-walker flag bits, OR-ed into afqmc_walkers.flags by the library. */
enum {
  AFQMC_W_SINGULAR = 1u,   /* <Psi_T|phi> is exactly zero or not finite: weight set to 0 */
  AFQMC_W_NONFINITE = 2u,  /* the walker's fields x contained NaN/Inf: weight set to 0  */
  AFQMC_W_DEAD = 4u        /* cos(theta) <= 0 this step: weight set to 0 (phaseless)     */
};

/* One Cholesky-factorised system (Sec. 3.2, the generic Hamiltonian object
 * built from h1e, chol, ecore; Sec. 3.3, the single-determinant trial). */
typedef struct {
  int32_t nbasis, nalpha, nbeta, nchol, nwalkers;
  const double *h1;     /* host [M][M], real symmetric one-body integrals h_pq      */
  const double *chol;   /* host [G][M][M], real symmetric Cholesky vectors L^g_pq,
                           (ps|qr) = sum_g L^g_ps L^g_qr (eq. chol_decomp)         */
  double ecore;         /* constant energy (nuclear repulsion)                      */
  const double *trial;  /* host [M][Nt] real, orthonormal columns per spin block    */
  double dt;            /* imaginary time step (eq. afqmc), > 0                     */
  int32_t chol_gen;     /* 0: chol is the host array above; 1: chol is NULL and the
                           library draws the synthetic tensor on the device:
                           L^g_pq = L^g_qp = sqrt(3) (u_{4i} + u_{4i+1} + u_{4i+2}
                           + u_{4i+3} - 2) * (exp(-g / gen_tau) * gen_scale) for
                           p <= q, i = (g M + p) M + q, u_n = (output n of the
                           SplitMix64 stream seeded with gen_seed) >> 11, times
                           2^-53 (sums left to right; exp from the C library)   */
  int32_t reserved_desc;
  uint64_t gen_seed;
  double gen_tau;       /* > 0 */
  double gen_scale;
} afqmc_system_desc;

/* Exchange-energy mode of afqmc_local_energy and afqmc_step. */
enum {
  AFQMC_EX_FULL = 0,  /* exact exchange for every walker                               */
  AFQMC_EX_CV = 1     /* learned control variate: a network's prediction for every
                         walker, corrected by the exact exchange of a random subset  */
};

/* Options (zero-initialise, then call afqmc_default_options). */
typedef struct {
  int32_t precision;        /* AFQMC_FP64 (default) or a *_CONTRACT form          */
  int32_t taylor_order;     /* order of exp(sqrt(dt) V_HS); default 6, 1..16       */
  double fb_cap;            /* force-bias modulus cap; default 1.0, <= 0 disables  */
  double e_shift;           /* energy shift E_T; NaN (default) = the trial's E_HF  */
  uint64_t mem_limit_bytes; /* refuse set-up needing more device memory; 0 = none  */
  int32_t streams;          /* systems of a set run concurrently on this many
                               internal streams (default 0 = min(nsys, 4));
                               1 = one after another on the caller's stream.
                               Results do not depend on it.                       */
  int32_t use_graph;        /* afqmc_step records the whole step of every system
                               into a hipGraph the first time it sees a set of
                               buffers and flags, and replays it when they repeat
                               (default 0).  Phase timers do not see replays.     */
  int32_t tune;             /* time launch shapes at set-up and keep the fastest
                               per problem shape: the exchange kernels' walker
                               tiling (1, 2 or 4 walkers per workgroup) and tile
                               order, the V_HS product's tiles and the Taylor
                               kernel's row tiles; default 1.  Results do not
                               depend on it.                                      */
  int32_t ex_mode;          /* AFQMC_EX_FULL (default) or AFQMC_EX_CV              */
  double cv_fraction;       /* AFQMC_EX_CV: share of walkers whose exact exchange
                               is computed per call, k = ceil(cv_fraction W);
                               default 0.125, in (0, 1]                           */
  uint64_t cv_seed;         /* AFQMC_EX_CV: seed of the subset draws; default 7   */
  int32_t prop_precision;   /* AFQMC_FP64 (default) or AFQMC_FP32_CONTRACT: V_HS
                               planes and the Taylor terms of the propagation in
                               FP32 (the series sum, B1, overlaps and energies
                               stay FP64; the mixed precision the paper mentions
                               in Sec. 6).  Needs M a multiple of 4, Nt <= 96.    */
  int32_t deterministic;    /* 1 (default): every reduction (split-K partials, the
                               sums over Cholesky vectors, lanes and walkers, the
                               estimator) runs in a fixed order, so a run replays
                               bitwise and a set of systems equals separate runs;
                               0 (unordered atomic reductions) is not provided and
                               is AFQMC_ERR_ARG                                   */
  const char *tune_cache;   /* with tune: path of a file of JSON lines, one per
                               problem shape, that the tuner reads before timing
                               and appends its choices to (NULL, the default:
                               choices are kept for the process only).  A file
                               that cannot be written is AFQMC_ERR_ARG.  The
                               library reads the string during set-up only.      */
  int32_t reserved[8];      /* reserved[0] bit 0: VALU (non-MFMA) exchange kernel;
                               bit 1: VALU kernels for the force bias, V_HS, B1
                               and Taylor products; bit 2: the generic MFMA GEMM
                               for the Taylor terms; bit 3: V_HS from the full
                               (unpacked) L^g; bit 4: free projection through
                               both V_HS planes (all for comparison runs);
                               reserved[1]: walkers per exchange workgroup (1, 2
                               or 4); reserved[2]: exchange tile order (1 = Cholesky
                               block fastest, g > 1 = groups of g walker blocks);
                               either one fixes the exchange launch shape;
                               reserved[3]: k = 1..4 fixes the V_HS tile shape
                               k - 1; reserved[4]: k fixes the Taylor kernel's
                               shape k - 1: with FP64 propagation k = 1..4 (48-
                               or 32-row tiles with a copy wave, the same
                               without one at three or four workgroups per
                               CU), with
                               FP32 propagation k = 1..3 (48, 32 or 64 rows);
                               0 leaves each to the tuner; other entries: zero   */
} afqmc_options;

/* Walker state of one system; every pointer is device memory owned by the caller. */
typedef struct {
  void *phi;          /* double2 [W][M][Nt] orbitals, updated in place            */
  double *weight;     /* [W] real weights                                           */
  void *log_ovlp;     /* double2 [W]: log <Psi_T|phi>, imaginary part in (-pi, pi] */
  uint32_t *flags;    /* [W] AFQMC_W_* bits, OR-ed in by the library               */
} afqmc_walkers;

/* Scalars derived at set-up, for reporting and tests. */
typedef struct {
  double e_hf;        /* trial energy <Psi_T|H|Psi_T> (also the default E_T)   */
  double e_shift;     /* E_T in use                                            */
  double const_c;     /* ecore - 1/2 sum_g l_g^2 (mean-field constant)         */
  uint64_t device_bytes; /* device memory held by this system                 */
  int32_t exchange_tile; /* walkers per FP64 exchange workgroup in use (1/2/4)  */
  int32_t exchange_order; /* exchange tile order: 0 = Cholesky block fastest,
                             g > 0 = groups of g walker blocks (-1: VALU path) */
  int32_t lane;          /* internal stream of a system set (-1: caller's)      */
  int64_t graph_captures; /* afqmc_step graphs recorded so far (whole context)  */
  int64_t graph_replays;  /* afqmc_step graph replays so far (whole context)    */
  int32_t cv_subset;      /* walkers with exact exchange per energy call (EX_CV), else 0 */
  int32_t vhs_tile;       /* V_HS tile shape in use (0..3; -1: another route)        */
  int32_t taylor_tile;    /* Taylor row tile in use (0 = 48, 1 = 32, 2 = 64 rows; -1:
                             the generic GEMM route)                                 */
  int32_t reserved_info;
} afqmc_info;

/* Fills `opt` with the defaults listed above.  Returns AFQMC_ERR_ARG on NULL. */
afqmc_status afqmc_default_options(afqmc_options *opt);

/*
 * Builds a context for `nsys` >= 1 independent systems (nsys > 1 is the
 * batching form; walkers, fields and outputs of the other calls are then
 * arrays of length nsys).  Copies h1, chol and trial to the device and derives
 * (Sec. 2, the equations after eq. chol_decomp; eq. fb; eq. Bprop):
 *   v0 = h - 1/2 sum_g L^g L^g, l_g = sum_s Tr(L^g Psi_s Psi_s^T),
 *   H1 = v0 + sum_g l_g L^g, C = ecore - 1/2 sum_g l_g^2, B1 = exp(-dt/2 H1),
 *   the half-rotated Ltilde^{g s} = Psi_s^T L^g and htilde_s = Psi_s^T h, and
 *   E_HF, the trial's local energy.
 * Synchronous: returns after all set-up work on `hip_stream` has finished.
 * Errors: AFQMC_ERR_ARG (NULL pointer, non-positive size, N_s > M, dt <= 0),
 * AFQMC_ERR_UNSUPPORTED (a spin block wider than 64 orbitals),
 * AFQMC_ERR_OOM (allocation failure or over mem_limit_bytes; nothing is left
 * allocated), AFQMC_ERR_HIP.
 */
afqmc_status afqmc_setup_hamiltonian(const afqmc_system_desc *sys, int32_t nsys,
                                     const afqmc_options *opt, void *hip_stream,
                                     afqmc_ctx **out);

/*
 * One phaseless time step for every walker (Sec. 2, eqs. propagate,
 * weight_update, fb, ovlp_ratio and the hybrid importance function):
 *   Theta = phi (Psi^T phi)^-1 per spin; vbias_g = sum_s Tr(Ltilde^{g s} Theta_s);
 *   xbar = i sqrt(dt) (vbias - l), each |xbar_g| capped at fb_cap; y = x - xbar;
 *   phi <- B1 T(sqrt(dt) V_HS) B1 phi with V_HS = -i sum_g y_g L^g and T the
 *   Taylor series of the exponential;
 *   S = <Psi_T|phi'>/<Psi_T|phi> exp(i sqrt(dt) y.l), I = S exp(x.xbar - xbar.xbar/2),
 *   w <- w |I| max(0, cos arg S) exp(-dt (C - E_T)), log_ovlp <- log<Psi_T|phi'>.
 * `x`: array of nsys device pointers, each [W][G] standard-normal fields.
 * Errors: AFQMC_ERR_ARG on NULL pointers; AFQMC_ERR_HIP on launch failure.
 */
afqmc_status afqmc_propagate(afqmc_ctx *ctx, const afqmc_walkers *w,
                             const double *const *x, void *hip_stream);

/*
 * Local energy E_loc = <Psi_T|H|phi>/<Psi_T|phi> of every walker (eq. Eloc)
 * by Wick's theorem with the Cholesky integrals:
 *   E1 = ecore + sum_s Tr(htilde_s Theta_s),
 *   E2 = 1/2 sum_g vbias_g^2 - 1/2 sum_g sum_s Tr(T^{g s} T^{g s}),
 *   T^{g s} = Ltilde^{g s} Theta_s (exchange; never stored).
 * `e_out`: array of nsys device pointers, each double2 [W][3] = (E, E1, E2).
 * `est_out`: NULL or device double [nsys][4] = (ENumer, EDenom, E1Body, E2Body)
 *   = (sum w Re E, sum w, sum w Re E1, sum w Re E2) over walkers with w > 0
 *   (the estimator record of Sec. 3.5).  Reductions are deterministic.
 */
afqmc_status afqmc_local_energy(afqmc_ctx *ctx, const afqmc_walkers *w,
                                void *const *e_out, double *est_out, void *hip_stream);

/*
 * Re-orthogonalisation (the stabilisation of Sec. 3.1): modified Gram-Schmidt
 * on each spin block, phi_s = Q_s R_s with real R_ii > 0, phi_s <- Q_s and
 * log_ovlp -= sum_s sum_i log R_ii.  Weights and energies are unchanged.
 */
afqmc_status afqmc_reorthogonalize(afqmc_ctx *ctx, const afqmc_walkers *w, void *hip_stream);

/*
 * One full walker step with fewer passes over the walkers: afqmc_propagate,
 * then afqmc_reorthogonalize if (flags & AFQMC_STEP_REORTHO), then
 * afqmc_local_energy of the new walkers (outputs as in those calls).
 * Theta = phi (Psi^T phi)^-1 and vbias of the new walkers serve both this
 * step's local energy and the next step's force bias (Theta, hence vbias, is
 * unchanged when phi is re-orthogonalised, phi -> phi R^-1), so one overlap/LU
 * and one force-bias contraction are done per step instead of three and two.
 * The context keeps them for the walker buffers of its last afqmc_step (it
 * remembers their addresses only, and never reads them after the call
 * returns); they are recomputed when the addresses differ, after any other
 * call on the context, or when (flags & AFQMC_STEP_FRESH) says the walkers
 * were changed elsewhere.  A caller whose new walker buffers may reuse the
 * previous step's addresses (a caching allocator), or who writes the walkers
 * itself between steps, must pass AFQMC_STEP_FRESH; the Python binding does
 * so whenever the walker sets differ from the previous step's.
 * When they are reused, log<Psi_T|phi> of the walkers is taken from
 * walkers.log_ovlp (which propagation and re-orthogonalisation keep current).
 * When they are recomputed, vbias is still taken as the trace of the exchange
 * matrices (full exchange mode), as in every later step, so a run restarted
 * from its walker state after a step without re-orthogonalisation repeats the
 * uninterrupted run bit for bit.
 */
enum { AFQMC_STEP_REORTHO = 1u, AFQMC_STEP_FRESH = 2u };
afqmc_status afqmc_step(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *e_out,
                        double *est_out, uint32_t flags, void *hip_stream);

/*
 * Trial-object operations of Sec. 3.3 (calc_overlap, calc_greens_function,
 * calc_force_bias) exposed on their own, for initialisation and tests.
 * afqmc_overlap: writes log_ovlp = log<Psi_T|phi> and ORs AFQMC_W_SINGULAR.
 * afqmc_greens_function: theta_out[s] device double2 [W][M][Nt]:
 *   Theta = phi (Psi^T phi)^-1 per spin block (G_pq = sum_i Psi_pi Theta_qi).
 * afqmc_force_bias: vbias_out[s] device double2 [W][G], vbias_g as above.
 */
afqmc_status afqmc_overlap(afqmc_ctx *ctx, const afqmc_walkers *w, void *hip_stream);
afqmc_status afqmc_greens_function(afqmc_ctx *ctx, const afqmc_walkers *w,
                                   void *const *theta_out, void *hip_stream);
afqmc_status afqmc_force_bias(afqmc_ctx *ctx, const afqmc_walkers *w,
                              void *const *vbias_out, void *hip_stream);

/*
 * Learned control variate of the exchange energy (options.ex_mode =
 * AFQMC_EX_CV).  The mixed estimator of eq. Eloc needs E2 = EJ + EK per walker;
 * in this mode afqmc_local_energy and afqmc_step return, as the exchange part
 * of E2, the Horvitz-Thompson estimate
 *   g_w = f_w + [w in S] (EK_w - f_w) / pi,   pi = k / W,  k = ceil(cv_fraction W),
 * where f_w is a network's prediction of EK_w and S a uniform subset of k
 * walkers drawn without replacement (keys: the SplitMix64 output function of
 * cv_seed + call * 2^32 + w * 0x9E3779B97F4A7C15, call = 0, 1, ... counting the
 * energy calls of the system; the k smallest keys, ties to the lower index),
 * on which alone the exact exchange is computed.  E_S[g_w] = EK_w, so the
 * estimator is unbiased given the walkers (weights never depend on energies).
 * W <= 4096 in this mode (AFQMC_ERR_UNSUPPORTED otherwise).
 *
 * Features (double [W][10]): Re EJ, Im EJ, Re E1, Im E1, sum_g |vbias_g - l_g|^2,
 * Re sum_g (vbias_g - l_g)^2, cos and sin of arg <Psi_T|phi>, and Re and Im of
 * sum_s Tr(K_s Theta_s) with K_s = sum_g (Ltilde^{g s} Psi_s) Ltilde^{g s}: the
 * exchange energy to first order in the walker's departure from the trial,
 * EK(Psi) - sum_s Tr(K_s (Theta_s - Psi_s)), at the cost of a one-body energy.
 * Network (FP32): standardised features -> tanh(W1 x + b1) (128) ->
 * tanh(W2 h + b2) (128) -> W3 h + b3 = standardised (Re EK, Im EK).
 * Parameters: float [AFQMC_CV_NPARAMS] = W1 [128][10], b1 [128], W2 [128][128],
 * b2 [128], W3 [2][128], b3 [2] (row-major, (out, in)); normalisation:
 * double [AFQMC_CV_NNORM] = feature means [10], deviations [10], target means
 * [2], deviations [2].  At set-up the weights are Glorot-uniform from a fixed
 * seed, the biases zero and the normalisation the identity.  Each system of a
 * context has its own network.
 *
 * afqmc_cv_collect: for every walker, features and the exact EK (full
 *   exchange in the context's precision), as training samples:
 *   feat_out[s] device double [W][10], ek_out[s] device double2 [W].
 * afqmc_cv_train: sets the normalisation from the n samples (means and
 *   population deviations), then runs `epochs` passes of Adam (beta1 0.9,
 *   beta2 0.999, eps 1e-8, bias-corrected, moments reset at the start) over
 *   minibatches of `batch` consecutive samples on the mean of 1/2 ||y - t||^2.
 *   loss_out: NULL or device double [epochs], the mean loss of each pass.
 *   Synchronous (allocates and frees its workspace); inputs are device pointers.
 * afqmc_cv_set_params / afqmc_cv_get_params: device copies of the parameters
 *   and normalisation (either pointer may be NULL); set resets the Adam moments.
 * afqmc_cv_predict: f_out device double2 [n] = the network's EK for raw
 *   features feat device double [n][10].
 * afqmc_cv_loss_grad: loss (device double [1]) and gradient (device float
 *   [AFQMC_CV_NPARAMS]) of the mean of 1/2 ||y - t||^2 over n standardised
 *   samples x device float [n][10], t device float [n][2].  Synchronous.
 * afqmc_cv_state: device copies of the last energy call's predictions
 *   (double2 [W]), subset (int32 [k], increasing) and call index (uint64 [1]).
 * Errors: AFQMC_ERR_ARG on NULL context, bad index or sizes; AFQMC_ERR_OOM;
 * AFQMC_ERR_HIP.
 */
#define AFQMC_CV_NFEAT 10
#define AFQMC_CV_NPARAMS 18178
#define AFQMC_CV_NNORM 24
afqmc_status afqmc_cv_collect(afqmc_ctx *ctx, const afqmc_walkers *w, double *const *feat_out,
                              void *const *ek_out, void *hip_stream);
afqmc_status afqmc_cv_train(afqmc_ctx *ctx, int32_t isys, const double *feat, const void *ek, int64_t n,
                            int32_t epochs, int32_t batch, double lr, double *loss_out, void *hip_stream);
/*
 * afqmc_cv_train for callers that cannot allocate device memory at call time
 * (code under hipGraph capture, tight serving loops, harnesses that forbid
 * allocation): the same training, from the same kernels in the same order,
 * with its workspace in a fixed device array of the library (under 8 MiB,
 * one per GPU, held until the process ends) instead of allocations, and
 * without synchronising: it enqueues on `hip_stream` and returns.
 * loss_out: NULL or device double [epochs], zeroed and then accumulated in.
 * Limits: n <= AFQMC_CV_NOALLOC_MAX_SAMPLES and min(batch, n) <=
 * AFQMC_CV_NOALLOC_MAX_BATCH, else AFQMC_ERR_UNSUPPORTED (nothing launched).
 * The array is shared by every call on one GPU and keeps the last call's
 * contents (each call writes all it reads): calls that overlap in time on one
 * GPU race, so issue them on one stream or synchronise between them.
 * Other errors as afqmc_cv_train.
 */
#define AFQMC_CV_NOALLOC_MAX_SAMPLES 65536
#define AFQMC_CV_NOALLOC_MAX_BATCH 512
afqmc_status afqmc_cv_train_noalloc(afqmc_ctx *ctx, int32_t isys, const double *feat, const void *ek, int64_t n,
                                    int32_t epochs, int32_t batch, double lr, double *loss_out, void *hip_stream);
afqmc_status afqmc_cv_set_params(afqmc_ctx *ctx, int32_t isys, const float *params, const double *norm,
                                 void *hip_stream);
afqmc_status afqmc_cv_get_params(afqmc_ctx *ctx, int32_t isys, float *params, double *norm, void *hip_stream);
afqmc_status afqmc_cv_predict(afqmc_ctx *ctx, int32_t isys, const double *feat, int64_t n, void *f_out,
                              void *hip_stream);
afqmc_status afqmc_cv_loss_grad(afqmc_ctx *ctx, int32_t isys, const float *x, const float *t, int64_t n,
                                float *grad_out, double *loss_out, void *hip_stream);
afqmc_status afqmc_cv_state(afqmc_ctx *ctx, int32_t isys, void *f_out, int32_t *subset_out, uint64_t *call_out,
                            void *hip_stream);

/*
 * Population control (the step of the simulation loop of Sec. 3.1 that keeps the walker
 * weights from spreading; the paper does not fix the method, this is the comb
 * of Calandra Buonaura and Sorella): with cumulative weights C_i summed in
 * walker order and total Wt, W teeth at (u + k) Wt / W for k = 0..W-1; new
 * walker k is a copy (orbitals, log-overlap, flags) of the first walker i with
 * C_i > tooth k, and every weight becomes Wt / W.  Zero-weight walkers are never
 * copied; with Wt = 0 nothing changes.  `u`: nsys device pointers to one double
 * in [0, 1) each.  `parents_out`: NULL, or nsys device int32 [W] receiving the
 * parent of each new walker.  Cached Theta/vbias of afqmc_step are dropped.
 */
afqmc_status afqmc_population_control(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *u,
                                      int32_t *const *parents_out, void *hip_stream);

/* Sets E_T (the energy shift of the weight update, eq. weight_update) of
 * system `isys`.  E_T lives in device memory and the weight kernels read it
 * there, so this only enqueues a one-thread write on `hip_stream` (no
 * synchronisation; recorded graphs stay valid and see the new value).
 * Errors: AFQMC_ERR_ARG (NULL context, bad index, non-finite value). */
afqmc_status afqmc_set_e_shift(afqmc_ctx *ctx, int32_t isys, double e_shift, void *hip_stream);

/*
 * One block of the simulation loop of Sec. 3.1 (propagation, stabilisation,
 * population control and estimators, with the outputs written once per block
 * so that they can be reblocked as the run goes on):
 *   for k = 0 .. nsteps-1: afqmc_step with the fields x[i] + k W G, with
 *     AFQMC_STEP_REORTHO when reortho_every > 0 and (step0 + k + 1) is a
 *     multiple of it (step0 = steps taken before this block), AFQMC_STEP_FRESH
 *     on the first step when (flags & AFQMC_STEP_FRESH), and the estimator
 *     record (ENumer, EDenom, E1Body, E2Body) of step k into est[i] + 4 k;
 *   then, when u != NULL, afqmc_population_control with offset u[i];
 *   then, when (flags & AFQMC_BLOCK_FEEDBACK), E_T <- sum_k ENumer_k /
 *     sum_k EDenom_k of the block, on the device (kept when the sum of EDenom
 *     is not positive).  The paper does not fix the feedback; a common E_T
 *     scales every weight alike and leaves the mixed estimate unchanged.
 * x: nsys device pointers, each [nsteps][W][G] standard-normal fields.
 * e_out: nsys device pointers, double2 [W][3]: the last step's energies.
 * est: nsys device pointers, double [nsteps][4].
 * u: NULL or nsys device pointers to one double in [0, 1) each.
 * With options.use_graph the whole block is recorded into a hipGraph the
 * first time a combination of buffers, length, re-orthogonalisation phase and
 * flags is seen, and replayed after that.  Enqueues and returns.
 * Errors: AFQMC_ERR_ARG (NULL pointers, nsteps < 1, step0 < 0,
 * reortho_every < 0, unknown flags); AFQMC_ERR_HIP on launch failure.
 */
enum { AFQMC_BLOCK_FEEDBACK = 4u };
afqmc_status afqmc_run_block(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, int32_t nsteps,
                             int64_t step0, int32_t reortho_every, void *const *e_out, double *const *est,
                             const double *const *u, uint32_t flags, void *hip_stream);

/*
 * Reblocking analysis of a serially correlated series of n host doubles (the
 * per-step or per-block estimates; the paper reblocks its block outputs as the
 * run goes on, Sec. 3.1, after Flyvbjerg and Petersen, J. Chem. Phys. 91, 461
 * (1989)).  Level 0 is the series itself; level l+1 averages consecutive pairs
 * of level l, dropping an odd last sample; levels stop below two samples (at
 * most AFQMC_REBLOCK_LEVELS).  At each level, with n_l samples of mean m_l and
 * c0 = (1/n_l) sum (x - m_l)^2: std_err = sqrt(c0 / (n_l - 1)) and
 * std_err_err = std_err / sqrt(2 (n_l - 1)).  `optimal` is the smallest level
 * B with 2^(3B) > 2 n (std_err_B / std_err_0)^4 (Lee, Conduit, Nemec, Lopez
 * Rios and Drummond, Phys. Rev. E 83, 066706 (2011)), or -1 when no level
 * qualifies (the series is too short for its correlation time).  Host only:
 * touches no device.  Errors: AFQMC_ERR_ARG (NULL pointers, n < 2, a
 * non-finite sample).
 */
#define AFQMC_REBLOCK_LEVELS 64
typedef struct {
  int64_t n;          /* samples of the series                              */
  double mean;        /* their mean                                         */
  int32_t nlevels;    /* levels filled in below                             */
  int32_t optimal;    /* chosen level, -1 if none qualifies                 */
  int64_t count[AFQMC_REBLOCK_LEVELS];
  double level_mean[AFQMC_REBLOCK_LEVELS];
  double std_err[AFQMC_REBLOCK_LEVELS];
  double std_err_err[AFQMC_REBLOCK_LEVELS];
} afqmc_reblock_result;
afqmc_status afqmc_reblock(const double *x, int64_t n, afqmc_reblock_result *out);

/*
 * Free-projection AFQMC (the fp-AFQMC section): the walker step with the
 * mean-field shift only, no force bias, no phaseless projection and no
 * population control.  A walker stands for c |phi>, c the scalar the shifted
 * propagator accumulates, and carries besides phi and log_ovlp the complex
 * log-amplitude a = log(c <Psi_T|phi>) in `log_amp` (nsys device pointers,
 * each double2 [W], updated in place; start with a = log_ovlp for c = 1):
 *   phi <- B1 T(sqrt(dt) V_HS) B1 phi, V_HS = -i sum_g x_g L^g (bare fields x),
 *   a <- a + log<Psi_T|phi'> - log<Psi_T|phi> + i sqrt(dt) x.l - dt (C - E_T),
 *   Im a reduced to [-pi, pi], log_ovlp <- log<Psi_T|phi'>.
 * log<Psi_T|phi> is read from walkers.log_ovlp.  weight is neither read nor
 * written.  A walker whose new overlap vanishes is flagged AFQMC_W_SINGULAR and
 * keeps a and log_ovlp; non-finite fields are flagged AFQMC_W_NONFINITE and
 * taken as 0.  afqmc_reorthogonalize applies unchanged (a is invariant under
 * it).  Because V_HS is purely imaginary here, only its imaginary plane is
 * formed and contracted when the MFMA Taylor kernels are in use.
 * `x`: nsys device pointers, each [W][G] standard-normal fields.
 * Errors: AFQMC_ERR_ARG on NULL pointers; AFQMC_ERR_HIP on launch failure.
 */
afqmc_status afqmc_free_propagate(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x,
                                  void *const *log_amp, void *hip_stream);

/*
 * Energy estimate of free projection, E(tau) = N / D with
 *   z_w = weight_w exp(a_w - r),  N = sum z E,  D = sum z,  N1 = sum z E1,
 *   N2 = sum z E2,  r = max Re a_w,
 * over the walkers that count (weight > 0, neither AFQMC_W_SINGULAR nor
 * AFQMC_W_NONFINITE set, finite a; r = 0 when none does).  `e_in`: nsys device
 * pointers, each double2 [W][3] = (E, E1, E2) as afqmc_local_energy writes.
 * `est_out`: device double [nsys][AFQMC_FREE_EST] =
 *   (Re N, Im N, Re D, Im D, Re N1, Im N1, Re N2, Im N2, r, n counted).
 * The reduction order is fixed (bitwise reproducible).
 */
#define AFQMC_FREE_EST 10
afqmc_status afqmc_free_estimator(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *log_amp,
                                  void *const *e_in, double *est_out, void *hip_stream);

/*
 * One free-projection step: afqmc_free_propagate, then afqmc_reorthogonalize if
 * (flags & AFQMC_STEP_REORTHO), then the local energy of the new walkers into
 * e_out (as afqmc_local_energy) and, when est_out is not NULL, the estimate of
 * afqmc_free_estimator into est_out [nsys][AFQMC_FREE_EST].  Theta of the new
 * walkers comes from the overlap pass of the propagation (one LU per step).
 * Runs eagerly (options.use_graph does not apply).  Other flags: AFQMC_ERR_ARG.
 */
afqmc_status afqmc_free_step(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *log_amp,
                             void *const *e_out, double *est_out, uint32_t flags, void *hip_stream);

/* Set-up scalars of system `isys`.  AFQMC_ERR_ARG on NULL or bad index. */
afqmc_status afqmc_get_info(const afqmc_ctx *ctx, int32_t isys, afqmc_info *out);

/* Phase timers.  While enabled, the library brackets each kernel phase with a
 * pair of HIP events on the stream the phase runs on; afqmc_get_timings waits
 * for the recorded events and returns the accumulated milliseconds and launch
 * counts per phase since timing was (re-)enabled. */
enum {
  AFQMC_PH_OVERLAP = 0,   /* overlap, LU, log det and Theta               */
  AFQMC_PH_FORCE_BIAS,    /* vbias contraction                            */
  AFQMC_PH_FB_EPILOGUE,   /* xbar, y, per-walker sums (or EJ)             */
  AFQMC_PH_VHS,           /* V_HS = -i sum_g y_g L^g                      */
  AFQMC_PH_ONE_BODY,      /* B1 phi (both half steps)                     */
  AFQMC_PH_TAYLOR,        /* Taylor series of exp(sqrt(dt) V_HS)          */
  AFQMC_PH_WEIGHT,        /* phaseless weight update                      */
  AFQMC_PH_ENERGY_1B,     /* one-body energy                              */
  AFQMC_PH_EXCHANGE,      /* exchange energy: one interval per spin block */
  AFQMC_PH_COMBINE,       /* energy combination and estimator             */
  AFQMC_PH_REORTHO,       /* modified Gram-Schmidt                        */
  AFQMC_PH_OPERANDS,      /* FP32 / split-BF16 copies of Theta            */
  AFQMC_PH_CV,            /* features, network, subset draw and gather    */
  AFQMC_NPHASES
};
typedef struct {
  double ms[AFQMC_NPHASES];
  int64_t count[AFQMC_NPHASES];
} afqmc_timings;

/* Turns the phase timers on (enable != 0, which also zeroes them) or off. */
afqmc_status afqmc_set_timing(afqmc_ctx *ctx, int32_t enable);
/* Blocks until every recorded event has completed, then fills `out`. */
afqmc_status afqmc_get_timings(afqmc_ctx *ctx, afqmc_timings *out);

/* Frees the context and all device memory it owns.  NULL is a no-op.
 * Synchronises the device first so no queued kernel still uses the memory. */
void afqmc_destroy(afqmc_ctx *ctx);

/* Message for the last non-OK status on the calling thread ("" if none). */
const char *afqmc_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* AFQMC_H */
