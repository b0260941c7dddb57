// C ABI of libafqmc: argument validation, set-up of the derived Hamiltonian on
// the device, and the enqueueing of the step kernels.  No exception crosses the
// boundary; every failure returns a status and records a thread-local message.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <map>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "afqmc_internal.h"

using namespace afqmc;

namespace {

thread_local std::string g_last_error;

afqmc_status fail(afqmc_status s, const std::string &msg) {
  g_last_error = msg;
  return s;
}

#define AFQMC_HIP(call, what)                                                                \
  do {                                                                                       \
    hipError_t e_ = (call);                                                                  \
    if (e_ != hipSuccess) return fail(AFQMC_ERR_HIP, std::string(what) + ": " + hipGetErrorString(e_)); \
  } while (0)

}  // namespace

namespace afqmc {
afqmc_status record_error(afqmc_status s, const char *msg) { return fail(s, msg); }
}  // namespace afqmc

namespace {

// Training workspace of afqmc_cv_train_noalloc: one fixed device array per GPU
// (standardised samples and targets, per-workgroup gradient partials, the
// gradient and the loss partials), so that the call allocates nothing.
constexpr int64_t kNoAllocMaxSamples = AFQMC_CV_NOALLOC_MAX_SAMPLES;
constexpr int kNoAllocMaxBatch = AFQMC_CV_NOALLOC_MAX_BATCH;
constexpr int kNoAllocMaxWg = (kNoAllocMaxBatch + kCvGradBlock - 1) / kCvGradBlock;
constexpr size_t pad256(size_t b) { return (b + 255) / 256 * 256; }
constexpr size_t kNaX = 0;
constexpr size_t kNaT = kNaX + pad256((size_t)kNoAllocMaxSamples * kCvFeatures * sizeof(float));
constexpr size_t kNaPart = kNaT + pad256((size_t)kNoAllocMaxSamples * 2 * sizeof(float));
constexpr size_t kNaGrad = kNaPart + pad256((size_t)kNoAllocMaxWg * kCvParams * sizeof(float));
constexpr size_t kNaLpart = kNaGrad + pad256((size_t)kCvParams * sizeof(float));
constexpr size_t kNoAllocBytes = kNaLpart + pad256((size_t)kNoAllocMaxWg * sizeof(double));
static_assert(kNoAllocBytes <= 8u << 20, "the no-allocation workspace stays under 8 MiB");

// In host code `scratch` names a host-side stand-in: its device address on
// each GPU comes from hipGetSymbolAddress (scratch_address) and only that
// address is ever handed to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

std::mutex g_scratch_mu;
std::map<int, unsigned char *> g_scratch_addr;  // device ordinal -> address of `scratch` there

// Looks up (once per device, with that device current, at context set-up) the
// device address of `scratch`.
afqmc_status bind_scratch(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_addr.count(device)) return AFQMC_OK;
  void *p = nullptr;
  hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
  if (e != hipSuccess || !p)
    return fail(AFQMC_ERR_HIP, std::string("address of the no-allocation workspace: ") + hipGetErrorString(e));
  g_scratch_addr[device] = static_cast<unsigned char *>(p);
  return AFQMC_OK;
}

unsigned char *scratch_address(int device) {
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  auto it = g_scratch_addr.find(device);
  return it == g_scratch_addr.end() ? nullptr : it->second;
}

}  // namespace

struct afqmc_ctx {
  std::vector<System> sys;
  Options opt;
  int device = 0;
  std::vector<void *> allocs;
  bool force_valu_exchange = false;  // reserved[0] & 1: use the VALU exchange kernel
  bool force_valu_gemm = false;      // reserved[0] & 2: VALU kernels for the other contractions
  int debug_bits = 0;                // reserved[0]
  int vhs_fixed = -1;                // reserved[3] - 1: V_HS tile shape fixed by the caller (-1: tuned)
  int taylor_fixed = -1;             // reserved[4] - 1: Taylor tile shape fixed by the caller (-1: tuned)
  std::string tune_cache;            // options.tune_cache ("" = none)
  int ex_wx = 2;                     // walkers per exchange workgroup (reserved[1]: 1, 2 or 4)
  int ex_group = 8;                  // exchange tile order (reserved[2]: 1 = plain, g > 1 = groups of g)
  bool ex_wx_forced = false;         // launch shape fixed by the caller: no tuning
  bool tune = true;
  // system sets: internal streams (default priority) the systems are spread
  // over, and the events that fork them from / join them into the caller's stream
  std::vector<hipStream_t> lanes;
  std::vector<int> lane_of;
  hipEvent_t fork_ev = nullptr;
  std::vector<hipEvent_t> join_ev;
  // graph replay of afqmc_step
  bool use_graph = false;
  bool capturing = false;
  hipStream_t cap_stream = nullptr;
  hipEvent_t g_in = nullptr, g_out = nullptr;
  struct GraphEntry {
    std::vector<uintptr_t> key;
    hipGraphExec_t exec;
  };
  std::vector<GraphEntry> graphs;  // most recent last
  int64_t graph_captures = 0, graph_replays = 0;
  // phase timers
  bool timing = false;
  std::vector<hipEvent_t> ev_start, ev_stop;
  std::vector<int> ev_phase;
  size_t ev_used = 0;
  double ph_ms[AFQMC_NPHASES] = {0};
  int64_t ph_count[AFQMC_NPHASES] = {0};
};

namespace {

// Folds every recorded event pair into the per-phase totals (waits for them).
void fold_timings(afqmc_ctx *c) {
  for (size_t i = 0; i < c->ev_used; ++i) {
    float ms = 0.0f;
    if (hipEventSynchronize(c->ev_stop[i]) == hipSuccess &&
        hipEventElapsedTime(&ms, c->ev_start[i], c->ev_stop[i]) == hipSuccess) {
      c->ph_ms[c->ev_phase[i]] += ms;
      c->ph_count[c->ev_phase[i]] += 1;
    }
  }
  c->ev_used = 0;
}

// Brackets one phase with events when timing is on.
struct Phase {
  afqmc_ctx *c;
  hipStream_t st;
  size_t slot = (size_t)-1;
  Phase(afqmc_ctx *c_, int phase, hipStream_t st_) : c(c_), st(st_) {
    if (!c || !c->timing || c->capturing) return;
    if (c->ev_used == 4096) fold_timings(c);
    if (c->ev_used == c->ev_start.size()) {
      hipEvent_t a, b;
      if (hipEventCreate(&a) != hipSuccess) return;
      if (hipEventCreate(&b) != hipSuccess) { (void)hipEventDestroy(a); return; }
      c->ev_start.push_back(a);
      c->ev_stop.push_back(b);
      c->ev_phase.push_back(0);
    }
    slot = c->ev_used++;
    c->ev_phase[slot] = phase;
    (void)hipEventRecord(c->ev_start[slot], st);
  }
  ~Phase() {
    if (slot != (size_t)-1) (void)hipEventRecord(c->ev_stop[slot], st);
  }
};

}  // namespace

namespace {

void free_all(afqmc_ctx *c) {
  for (void *p : c->allocs)
    if (p) (void)hipFree(p);
  c->allocs.clear();
}

// Frees one allocation of the context (the device must be done with it).
void free_one(afqmc_ctx *c, void *p) {
  for (size_t i = 0; i < c->allocs.size(); ++i)
    if (c->allocs[i] == p) {
      (void)hipFree(p);
      c->allocs.erase(c->allocs.begin() + (long)i);
      return;
    }
}

// Releases everything the context holds (after the device has finished with it).
void release(afqmc_ctx *c) {
  (void)hipDeviceSynchronize();
  for (auto &g : c->graphs) (void)hipGraphExecDestroy(g.exec);
  c->graphs.clear();
  for (hipStream_t l : c->lanes) (void)hipStreamDestroy(l);
  c->lanes.clear();
  for (System &sy : c->sys) {
    if (sy.half_stream) (void)hipStreamDestroy(sy.half_stream);
    for (hipEvent_t e : {sy.half_fork, sy.half_join})
      if (e) (void)hipEventDestroy(e);
    sy.half_stream = nullptr;
    sy.half_fork = sy.half_join = nullptr;
  }
  for (hipEvent_t e : c->join_ev) (void)hipEventDestroy(e);
  c->join_ev.clear();
  for (hipEvent_t e : {c->fork_ev, c->g_in, c->g_out})
    if (e) (void)hipEventDestroy(e);
  c->fork_ev = c->g_in = c->g_out = nullptr;
  if (c->cap_stream) (void)hipStreamDestroy(c->cap_stream);
  c->cap_stream = nullptr;
  for (hipEvent_t e : c->ev_start) (void)hipEventDestroy(e);
  for (hipEvent_t e : c->ev_stop) (void)hipEventDestroy(e);
  c->ev_start.clear();
  c->ev_stop.clear();
  free_all(c);
}

// Device allocation recorded in the context; returns false on failure.
template <class T>
bool dalloc(afqmc_ctx *c, T **p, size_t count) {
  void *q = nullptr;
  if (count == 0) count = 1;
  if (hipMalloc(&q, count * sizeof(T)) != hipSuccess) {
    (void)hipGetLastError();
    *p = nullptr;
    return false;
  }
  c->allocs.push_back(q);
  *p = static_cast<T *>(q);
  return true;
}

// Set-up temporaries: freed (after a stream synchronisation) when the holder dies.
struct Temps {
  std::vector<void *> ptrs;
  hipStream_t st = nullptr;
  ~Temps() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(st);
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  bool get(T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    ptrs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
  }
};

bool valid_desc(const afqmc_system_desc &d, std::string &why) {
  if (d.chol_gen != 0 && d.chol_gen != 1) { why = "chol_gen must be 0 or 1"; return false; }
  if (!d.h1 || !d.trial || (d.chol_gen == 0 && !d.chol)) {
    why = "h1, trial and (unless chol_gen = 1) chol must be non-NULL host pointers";
    return false;
  }
  if (d.chol_gen == 1 && !(d.gen_tau > 0.0 && std::isfinite(d.gen_tau) && std::isfinite(d.gen_scale))) {
    why = "gen_tau must be positive and finite, gen_scale finite";
    return false;
  }
  if (d.nbasis <= 0 || d.nchol <= 0 || d.nwalkers <= 0) { why = "nbasis, nchol and nwalkers must be positive"; return false; }
  if (d.nalpha < 0 || d.nbeta < 0 || d.nalpha + d.nbeta <= 0) { why = "need at least one electron"; return false; }
  if (d.nalpha > d.nbasis || d.nbeta > d.nbasis) { why = "more electrons of one spin than orbitals"; return false; }
  if (!(d.dt > 0.0) || !std::isfinite(d.dt)) { why = "dt must be positive and finite"; return false; }
  if (!std::isfinite(d.ecore)) { why = "ecore must be finite"; return false; }
  return true;
}

// Sizes of every buffer of one system (doubles, double2s, uint32s).
struct Plan {
  size_t L, LtT, htT, trial, B1, lmf, theta, fbpart, yp, vhs, tbuf, wsc, wvec2, ekpart, stat, LtS0, LtS1, Lp, vhsp;
  size_t vhs32, t32;  // FP32 propagation: floats, complex floats
  size_t lp_bytes[2][2];  // reduced-precision operands per spin: [lhs, rhs] in bytes
  uint64_t bytes() const {
    return 8ull * (L + LtT + htT + trial + B1 + lmf + yp + vhs + wsc + LtS0 + LtS1 + Lp + vhsp) +
           16ull * (theta + fbpart + 3 * tbuf + 5 * wvec2 + ekpart + 2 * stat) + 4ull * 4 * stat + 4ull * vhs32 +
           16ull * t32 +
           lp_bytes[0][0] +
           lp_bytes[0][1] + lp_bytes[1][0] + lp_bytes[1][1];
  }
};

Plan plan_for(const System &s) {
  Plan p{};
  const size_t M = s.M, Nt = s.Nt, G = s.G, W = s.W;
  p.L = G * M * M;
  p.LtT = G * M * Nt;
  p.htT = M * Nt;
  p.trial = M * Nt;
  p.B1 = M * M;
  p.lmf = G;
  p.theta = W * M * Nt;
  p.fbpart = (size_t)std::max(s.fb_ksplit, 2) * W * G;
  p.yp = 2 * W * G;
  p.vhs = s.prop32 ? 0 : 2 * W * M * M;
  p.vhs32 = s.prop32 ? 2 * W * M * M : 0;
  p.t32 = s.prop32 ? W * M * Nt : 0;
  p.Lp = s.pack_chol ? G * (M * (M + 1) / 2) : 0;
  p.vhsp = s.pack_chol ? 2 * W * (M * (M + 1) / 2) : 0;
  p.tbuf = W * M * Nt;
  p.wsc = 6 * W;
  p.wvec2 = W;  // logo_now, logo_new, e1, ej (+1 spare)
  p.ekpart = W * 2 * (size_t)s.ex_stride;
  p.LtS0 = s.ex_mfma && s.Na > 0 ? G * M * (size_t)s.ex_plan[0].NR : 0;
  p.LtS1 = s.ex_mfma && s.Nb > 0 ? G * M * (size_t)s.ex_plan[1].NR : 0;
  for (int sp = 0; sp < 2; ++sp) {
    const bool on = s.precision != AFQMC_FP64 && s.ex_plan[sp].N > 0;
    p.lp_bytes[sp][0] = on ? lp_operand_bytes(s.precision, s.G, s.M, s.W, s.ex_plan[sp].NR, true) : 0;
    p.lp_bytes[sp][1] = on ? lp_operand_bytes(s.precision, s.G, s.M, s.W, s.ex_plan[sp].NR, false) : 0;
  }
  p.stat = W;
  return p;
}

int choose_fb_ksplit(int W, int G, long K) {
  // 64 x 64 output tiles over (2W rows) x (G columns)
  const long tiles = (long)((2 * W + 63) / 64) * ((G + 63) / 64);
  long ks = (1024 + tiles - 1) / tiles;
  ks = std::min(ks, std::max(1L, K / 512));
  return (int)std::max(1L, std::min(ks, 64L));
}

// Exchange energy of `W` walkers whose Theta is in `theta` (contiguous), into
// the partial sums s.ekpart; vbpart as in launch_exchange.
afqmc_status exchange_sys(afqmc_ctx *c, System &s, const double2 *theta, int W, double2 *vbpart, hipStream_t st) {
  for (int spin = 0; spin < 2; ++spin) {
    if (s.precision != AFQMC_FP64) {
      {
        Phase ph(c, AFQMC_PH_OPERANDS, st);
        AFQMC_HIP(lp_prepare_rhs(s, theta, W, spin, st), "reduced-precision operand kernel");
      }
      Phase ph(c, AFQMC_PH_EXCHANGE, st);
      AFQMC_HIP(launch_exchange_lp(s, W, spin, st, vbpart), "reduced-precision exchange kernel");
    } else {
      Phase ph(c, AFQMC_PH_EXCHANGE, st);
      AFQMC_HIP(launch_exchange(s, theta, W, st, vbpart, spin), "exchange kernel");
    }
  }
  return AFQMC_OK;
}

// Local energy in the control-variate mode (Theta of the walkers in s.theta,
// overlaps in s.logo_new): vbias by its own contraction, E1, EJ, features,
// network, subset draw, exact exchange of the subset, Horvitz-Thompson combine.
afqmc_status cv_energy_sys(afqmc_ctx *c, System &s, int W, double2 *e_out, double *est, const double *weight,
                           hipStream_t st) {
  {
    Phase ph(c, AFQMC_PH_FORCE_BIAS, st);
    AFQMC_HIP(launch_force_bias_gemm(s, s.theta, W, st), "force-bias kernel");
  }
  s.fb_slices = s.fb_ksplit;
  {
    Phase ph(c, AFQMC_PH_ENERGY_1B, st);
    AFQMC_HIP(launch_energy_e1(s, s.theta, W, st), "one-body energy kernel");
  }
  {
    Phase ph(c, AFQMC_PH_FB_EPILOGUE, st);
    AFQMC_HIP(launch_fb_energy_epilogue(s, W, nullptr, s.fb_slices, st), "Coulomb epilogue");
  }
  {
    Phase ph(c, AFQMC_PH_CV, st);
    AFQMC_HIP(launch_cv_features(s, W, s.cv_feat, st), "feature kernel");
    AFQMC_HIP(launch_cv_predict(s, s.cv_feat, W, s.cv_f, st), "network kernel");
    AFQMC_HIP(launch_cv_subset(s, W, s.cv_k, s.cv_seed, st), "subset kernel");
    AFQMC_HIP(launch_cv_gather(s, s.cv_k, st), "gather kernel");
  }
  afqmc_status r = exchange_sys(c, s, s.cv_theta, s.cv_k, nullptr, st);
  if (r != AFQMC_OK) return r;
  {
    Phase ph(c, AFQMC_PH_COMBINE, st);
    AFQMC_HIP(launch_cv_combine(s, W, s.cv_k, e_out, st), "energy combine kernel");
    if (est) AFQMC_HIP(launch_estimator(weight, e_out, W, est, st), "estimator kernel");
  }
  return AFQMC_OK;
}

// Local energy of W walkers of system s into e_out (device double2 [W][3]).
// `c` may be NULL (set-up); it only supplies the phase timers.
afqmc_status local_energy_sys(afqmc_ctx *c, System &s, const double2 *phi, int W, double2 *e_out, double *est,
                              const double *weight, hipStream_t st, bool have_theta = false) {
  if (!have_theta) {
    Phase ph(c, AFQMC_PH_OVERLAP, st);
    AFQMC_HIP(launch_ovlp_theta(phi, s.trial, s.M, s.Na, s.Nb, W, s.theta, s.logo_new, s.stat_new, nullptr, st, s.opart, s.ospart),
              "overlap kernel");
  }
  if (s.ex_mode == AFQMC_EX_CV && W == s.W) return cv_energy_sys(c, s, W, e_out, est, weight, st);
  // vbias: as the trace of the exchange matrices (MFMA exchange), else by its own contraction
  const bool fused_vb = s.ex_mfma;
  if (!fused_vb) {
    {
      Phase ph(c, AFQMC_PH_FORCE_BIAS, st);
      AFQMC_HIP(launch_force_bias_gemm(s, s.theta, W, st), "force-bias kernel");
    }
    s.fb_slices = s.fb_ksplit;
  }
  {
    Phase ph(c, AFQMC_PH_ENERGY_1B, st);
    AFQMC_HIP(launch_energy_e1(s, s.theta, W, st), "one-body energy kernel");
  }
  {
    afqmc_status r = exchange_sys(c, s, s.theta, W, fused_vb ? s.fbpart : nullptr, st);
    if (r != AFQMC_OK) return r;
  }
  if (fused_vb) s.fb_slices = 2;
  {
    Phase ph(c, AFQMC_PH_FB_EPILOGUE, st);
    AFQMC_HIP(launch_fb_energy_epilogue(s, W, nullptr, s.fb_slices, st), "Coulomb epilogue");
  }
  {
    Phase ph(c, AFQMC_PH_COMBINE, st);
    AFQMC_HIP(launch_energy_combine(s, W, e_out, st), "energy combine kernel");
    if (est) AFQMC_HIP(launch_estimator(weight, e_out, W, est, st), "estimator kernel");
  }
  return AFQMC_OK;
}

// exp(f X) for a real M x M device matrix X by a degree-20 Taylor series with
// scaling and squaring: f X is scaled by 2^-k until its 1-norm is at most 1/2
// (truncation error below 1e-22 relative), then squared k times.
afqmc_status device_expm(Temps &t, const double *X, double f, double xnorm1, int M, double *out,
                         hipStream_t st) {
  int sq = 0;
  double nrm = std::fabs(f) * xnorm1;
  while (nrm > 0.5) {
    nrm *= 0.5;
    ++sq;
  }
  const double scale = f * std::ldexp(1.0, -sq);
  double *term = nullptr, *tmp = nullptr, *xs = nullptr;
  const size_t mm = (size_t)M * M;
  if (!t.get(&term, mm) || !t.get(&tmp, mm) || !t.get(&xs, mm))
    return fail(AFQMC_ERR_OOM, "device allocation failed (matrix exponential)");
  AFQMC_HIP(hipMemsetAsync(out, 0, mm * sizeof(double), st), "memset");
  AFQMC_HIP(launch_add_identity(out, M, 1.0, st), "identity");
  AFQMC_HIP(hipMemsetAsync(xs, 0, mm * sizeof(double), st), "memset");
  AFQMC_HIP(launch_axpby(X, scale, xs, 0.0, (long)mm, st), "scale");
  AFQMC_HIP(hipMemcpyAsync(term, xs, mm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  AFQMC_HIP(launch_axpby(term, 1.0, out, 1.0, (long)mm, st), "axpy");
  for (int k = 2; k <= 20; ++k) {
    GemmArgs g;
    g.m = M; g.n = M; g.k = M;
    g.A = term; g.sai = M; g.sak = 1;
    g.B = xs; g.sbk = M; g.sbj = 1;
    g.C = tmp; g.sci = M; g.scj = 1;
    g.alpha = 1.0 / k;
    AFQMC_HIP(gemm_f64(g, st), "expm gemm");
    std::swap(term, tmp);
    AFQMC_HIP(launch_axpby(term, 1.0, out, 1.0, (long)mm, st), "axpy");
  }
  for (int k = 0; k < sq; ++k) {
    GemmArgs g;
    g.m = M; g.n = M; g.k = M;
    g.A = out; g.sai = M; g.sak = 1;
    g.B = out; g.sbk = M; g.sbj = 1;
    g.C = tmp; g.sci = M; g.scj = 1;
    AFQMC_HIP(gemm_f64(g, st), "expm squaring");
    AFQMC_HIP(hipMemcpyAsync(out, tmp, mm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  }
  return AFQMC_OK;
}

afqmc_status setup_one(afqmc_ctx *c, const afqmc_system_desc &d, System &s, hipStream_t st,
                       uint64_t *bytes_used, uint64_t limit) {
  s.M = d.nbasis; s.Na = d.nalpha; s.Nb = d.nbeta; s.Nt = d.nalpha + d.nbeta; s.G = d.nchol;
  s.W = d.nwalkers; s.dt = d.dt; s.sqdt = std::sqrt(d.dt); s.ecore = d.ecore;
  const int nmax = std::max(s.Na, s.Nb);
  if (nmax > kMaxSpinOrbitals)
    return fail(AFQMC_ERR_UNSUPPORTED, "a spin block wider than " + std::to_string(kMaxSpinOrbitals) +
                                           " orbitals is not supported");
  s.use_mfma_gemm = !c->force_valu_gemm;
  s.taylor_kernel = !(c->debug_bits & 4);
  s.vhs_shape = std::max(c->vhs_fixed, 0);
  s.taylor_shape = std::max(c->taylor_fixed, 0);
  s.pack_chol = s.use_mfma_gemm && !(c->debug_bits & 8);
  s.free_full = (c->debug_bits & 16) != 0;
  s.prop32 = c->opt.prop_precision == AFQMC_FP32_CONTRACT;
  if (s.prop32 && !(s.pack_chol && prop32_supported(s.M, s.Nt)))
    return fail(AFQMC_ERR_UNSUPPORTED, "FP32 propagation needs the MFMA path, M a multiple of 4 and at most 96 "
                                       "electrons");
  s.precision = c->opt.precision;
  s.fb_ksplit = choose_fb_ksplit(s.W, s.G, (long)s.M * s.Nt);
  exchange_geometry(nmax, &s.ex_gb, &s.ex_lds);
  s.ex_ngb = (s.G + s.ex_gb - 1) / s.ex_gb;
  s.ex_plan[0] = exchange_plan(s.Na, s.G, c->ex_wx);
  s.ex_plan[1] = exchange_plan(s.Nb, s.G, c->ex_wx);
  s.ex_group = c->ex_group;
  s.ex_mfma = (s.Na == 0 || s.ex_plan[0].mfma) && (s.Nb == 0 || s.ex_plan[1].mfma) && !c->force_valu_exchange;
  if (s.precision != AFQMC_FP64) {
    const bool ok = s.ex_mfma && (s.Na == 0 || lp_exchange_supported(s.precision, s.ex_plan[0].NR)) &&
                    (s.Nb == 0 || lp_exchange_supported(s.precision, s.ex_plan[1].NR));
    if (!ok) return fail(AFQMC_ERR_UNSUPPORTED, "reduced precision is built for spin blocks of up to 48 orbitals");
    for (int sp = 0; sp < 2; ++sp)
      if ((sp ? s.Nb : s.Na) > 0 && !lp_operands_addressable(s.precision, s.G, s.M, s.W, s.ex_plan[sp].NR))
        return fail(AFQMC_ERR_UNSUPPORTED, "reduced-precision exchange operands exceed 2^32 elements");
  }
  if (s.ex_mfma) {
    s.ex_nparts[0] = s.ex_plan[0].ngroups;
    s.ex_nparts[1] = s.ex_plan[1].ngroups;
    s.ex_stride = std::max(1, std::max(s.ex_nparts[0], s.ex_nparts[1]));
  } else {
    s.ex_nparts[0] = s.ex_nparts[1] = s.ex_stride = s.ex_ngb;
  }
  const Plan p = plan_for(s);
  const size_t M = s.M, Nt = s.Nt, G = s.G;
  const uint64_t setup_tmp = 8ull * (4 * M * M + M * M * 64 + M * M + G) + 16ull * (M * Nt + 3);
  s.bytes = p.bytes() + 8;
  if (limit && *bytes_used + s.bytes + setup_tmp > limit)
    return fail(AFQMC_ERR_OOM, "device memory needed (" + std::to_string(*bytes_used + s.bytes + setup_tmp) +
                                   " bytes) exceeds mem_limit_bytes");
  bool ok = dalloc(c, &s.eshift, 1) && dalloc(c, &s.L, p.L) && dalloc(c, &s.LtT, p.LtT) && dalloc(c, &s.htT, p.htT) &&
            dalloc(c, &s.trial, p.trial) && dalloc(c, &s.B1, p.B1) && dalloc(c, &s.lmf, p.lmf) &&
            dalloc(c, &s.theta, p.theta) && dalloc(c, &s.fbpart, p.fbpart) && dalloc(c, &s.yp, p.yp) &&
            (p.vhs == 0 || dalloc(c, &s.vhs, p.vhs)) && dalloc(c, &s.tA, p.tbuf) && dalloc(c, &s.tB, p.tbuf) &&
            (p.vhs32 == 0 || (dalloc(c, &s.vhs32, p.vhs32) && dalloc(c, &s.tA32, p.t32) &&
                              dalloc(c, &s.tB32, p.t32))) &&
            dalloc(c, &s.tacc, p.tbuf) && dalloc(c, &s.wsc, p.wsc) && dalloc(c, &s.logo_now, p.wvec2) &&
            dalloc(c, &s.logo_new, p.wvec2) && dalloc(c, &s.e1, p.wvec2) && dalloc(c, &s.ej, p.wvec2) &&
            dalloc(c, &s.ekpart, p.ekpart) && dalloc(c, &s.stat_now, p.stat) && dalloc(c, &s.stat_new, p.stat) &&
            dalloc(c, &s.opart, 2 * p.stat) && dalloc(c, &s.ospart, 2 * p.stat) &&
            (p.LtS0 == 0 || dalloc(c, &s.LtS[0], p.LtS0)) && (p.LtS1 == 0 || dalloc(c, &s.LtS[1], p.LtS1)) &&
            (p.Lp == 0 || (dalloc(c, &s.Lp, p.Lp) && dalloc(c, &s.vhsp, p.vhsp)));
  for (int sp = 0; sp < 2 && ok; ++sp) {
    unsigned char *b0 = nullptr, *b1 = nullptr;
    if (p.lp_bytes[sp][0]) ok = ok && dalloc(c, &b0, p.lp_bytes[sp][0]) && dalloc(c, &b1, p.lp_bytes[sp][1]);
    s.lp_lhs[sp] = b0;
    s.lp_rhs[sp] = b1;
  }
  // learned control variate: network state (small) always, Theta of the subset in EX_CV mode
  s.cv_seed = c->opt.cv_seed;
  s.cv_k = (int)std::min<double>(s.W, std::max(1.0, std::ceil(c->opt.cv_fraction * s.W - 1e-9)));
  {
    const size_t Wn = s.W;
    ok = ok && dalloc(c, &s.cv_params, kCvParams) && dalloc(c, &s.cv_m, kCvParams) &&
         dalloc(c, &s.cv_v, kCvParams) && dalloc(c, &s.cv_norm, kCvNorm) &&
         dalloc(c, &s.cv_feat, Wn * kCvFeatures) && dalloc(c, &s.cv_f, Wn) && dalloc(c, &s.cv_sel, Wn) &&
         dalloc(c, &s.cv_pos, Wn) && dalloc(c, &s.cv_counter, 2) && dalloc(c, &s.KtT, M * Nt) &&
         dalloc(c, &s.cv_lin, Wn);
    if (ok && c->opt.ex_mode == AFQMC_EX_CV) ok = dalloc(c, &s.cv_theta, (size_t)s.cv_k * M * Nt);
    s.bytes += 4ull * 3 * kCvParams + 8ull * (kCvNorm + Wn * kCvFeatures) + 16ull * Wn + 8ull * Wn + 16 +
               8ull * M * Nt + 16ull * Wn +
               (c->opt.ex_mode == AFQMC_EX_CV ? 16ull * s.cv_k * M * Nt : 0);
  }
  if (!ok) return fail(AFQMC_ERR_OOM, "device allocation failed");
  *bytes_used += s.bytes;
  AFQMC_HIP(cv_enable_lds(), "network kernel LDS attribute");
  AFQMC_HIP(launch_cv_init(s, 0x5EEDull, st), "network initialisation");
  AFQMC_HIP(launch_cv_zero(s.cv_m, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(s.cv_v, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(s.cv_counter, 2 * sizeof(uint64_t), st), "zero fill");
  AFQMC_HIP(exchange_enable_lds(s), "exchange kernel LDS attribute");
  AFQMC_HIP(ovlp_enable_lds(nmax), "overlap kernel LDS attribute");
  if (s.precision != AFQMC_FP64) AFQMC_HIP(lp_enable_lds(s), "reduced-precision exchange LDS attribute");

  const size_t mm = M * M;
  if (d.chol_gen == 1) {
    std::vector<double> fac(G);
    for (size_t g = 0; g < G; ++g) fac[g] = std::exp(-(double)g / d.gen_tau) * d.gen_scale;
    double *dfac = nullptr;
    Temps gt;
    gt.st = st;
    if (!gt.get(&dfac, G)) return fail(AFQMC_ERR_OOM, "device allocation failed (generator factors)");
    AFQMC_HIP(hipMemcpyAsync(dfac, fac.data(), G * sizeof(double), hipMemcpyHostToDevice, st), "upload factors");
    AFQMC_HIP(launch_gen_chol(s, d.gen_seed, dfac, std::sqrt(3.0), st), "Cholesky generator");
  } else {
    AFQMC_HIP(hipMemcpyAsync(s.L, d.chol, p.L * sizeof(double), hipMemcpyHostToDevice, st), "upload chol");
  }
  if (s.Lp) AFQMC_HIP(launch_pack_upper(s, st), "Cholesky packing");
  if (s.prop32) {
    // FP32 propagation forms V_HS in FP32 from an FP32 copy of the packed vectors
    const long Mp = (long)M * (M + 1) / 2;
    s.ldlp32 = (Mp + 3) / 4 * 4;
    if (!dalloc(c, &s.Lp32, (size_t)G * s.ldlp32)) return fail(AFQMC_ERR_OOM, "device allocation failed (FP32 L)");
    s.bytes += 4ull * G * s.ldlp32;
    AFQMC_HIP(launch_pack_to_f32(s.Lp, Mp, G, s.ldlp32, s.Lp32, st), "FP32 packed Cholesky vectors");
  }
  AFQMC_HIP(hipMemcpyAsync(s.trial, d.trial, p.trial * sizeof(double), hipMemcpyHostToDevice, st),
            "upload trial");
  // temporaries of set-up
  Temps tmp;
  tmp.st = st;
  double *h = nullptr, *P = nullptr, *v0 = nullptr, *H1 = nullptr, *parts = nullptr;
  const int tiles = (int)(((M + 63) / 64) * ((M + 63) / 64));
  const long Kx = (long)G * M;
  int ksx = std::max(1, std::min((1024 + tiles - 1) / tiles, (int)std::max(1L, Kx / 256)));
  ksx = std::min(ksx, 64);
  if (!tmp.get(&h, mm) || !tmp.get(&P, mm) || !tmp.get(&v0, mm) || !tmp.get(&H1, mm) ||
      !tmp.get(&parts, (size_t)ksx * mm))
    return fail(AFQMC_ERR_OOM, "device allocation failed (set-up temporaries)");
  AFQMC_HIP(hipMemcpyAsync(h, d.h1, mm * sizeof(double), hipMemcpyHostToDevice, st), "upload h1");
  // trial density matrix P = sum_s Psi_s Psi_s^T (host)
  std::vector<double> hP(mm, 0.0);
  for (size_t pp = 0; pp < M; ++pp)
    for (size_t qq = 0; qq < M; ++qq) {
      double a = 0.0;
      for (size_t i = 0; i < Nt; ++i) a += d.trial[pp * Nt + i] * d.trial[qq * Nt + i];
      hP[pp * M + qq] = a;
    }
  AFQMC_HIP(hipMemcpyAsync(P, hP.data(), mm * sizeof(double), hipMemcpyHostToDevice, st), "upload P");
  // l_g = sum_pq L^g_pq P_pq
  AFQMC_HIP(launch_row_dot(s.L, P, (long)mm, s.G, s.lmf, st), "mean-field shift");
  // v0 = h - 1/2 sum_g L^g L^g; with L viewed as a (G M) x M matrix B, sum_g L^g L^g = B^T B
  {
    GemmArgs g;
    g.m = s.M; g.n = s.M; g.k = (int)Kx; g.ksplit = ksx;
    g.A = s.L; g.sai = 1; g.sak = s.M;
    g.B = s.L; g.sbk = s.M; g.sbj = 1;
    g.C = parts; g.sci = s.M; g.scj = 1; g.scs = (long)mm;
    AFQMC_HIP(gemm_f64(g, st), "v0 gemm");
    AFQMC_HIP(hipMemcpyAsync(v0, h, mm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
    AFQMC_HIP(launch_sum_slices(parts, ksx, (long)mm, -0.5, v0, st), "v0 reduce");
  }
  // H1 = v0 + sum_g l_g L^g
  {
    AFQMC_HIP(hipMemcpyAsync(H1, v0, mm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
    GemmArgs g;
    g.m = 1; g.n = (int)mm; g.k = s.G;
    g.A = s.lmf; g.sai = 0; g.sak = 1;
    g.B = s.L; g.sbk = (long)mm; g.sbj = 1;
    g.C = H1; g.sci = 0; g.scj = 1; g.beta = 1.0;
    AFQMC_HIP(gemm_f64(g, st), "H1 gemm");
  }
  // half rotation: LtT[g] = L^g Psi (= (Psi^T L^g)^T), htT = h Psi
  {
    GemmArgs g;
    g.m = s.M; g.n = s.Nt; g.k = s.M; g.batch = s.G;
    g.A = s.L; g.sai = s.M; g.sak = 1; g.sab = (long)mm;
    g.B = s.trial; g.sbk = s.Nt; g.sbj = 1; g.sbb = 0;
    g.C = s.LtT; g.sci = s.Nt; g.scj = 1; g.scb = (long)M * Nt;
    AFQMC_HIP(gemm_f64(g, st), "half-rotation gemm");
    GemmArgs gh = g;
    gh.batch = 1; gh.A = h; gh.sab = 0; gh.C = s.htT; gh.scb = 0;
    AFQMC_HIP(gemm_f64(gh, st), "half-rotation of h");
    for (int sp = 0; sp < 2; ++sp)
      if (s.LtS[sp])
        AFQMC_HIP(launch_pad_half_rotated(s.LtT, s.G, s.M, s.Nt, sp ? s.Na : 0, sp ? s.Nb : s.Na,
                                          s.ex_plan[sp].NR, s.LtS[sp], st),
                  "padded half rotation");
    for (int sp = 0; sp < 2; ++sp)
      if (s.lp_lhs[sp]) AFQMC_HIP(lp_prepare_lhs(s, sp, st), "reduced-precision half rotation");
    // K_s of the control variate's first-order exchange feature
    double *t0 = nullptr;
    if (!tmp.get(&t0, G * Nt * Nt)) return fail(AFQMC_ERR_OOM, "device allocation failed (first-order exchange)");
    AFQMC_HIP(launch_cv_kmat(s, t0, st), "first-order exchange matrices");
  }
  // scalars and B1 = exp(-dt/2 H1)
  std::vector<double> hl(G), hH1(mm);
  AFQMC_HIP(hipMemcpyAsync(hl.data(), s.lmf, G * sizeof(double), hipMemcpyDeviceToHost, st), "download l");
  AFQMC_HIP(hipMemcpyAsync(hH1.data(), H1, mm * sizeof(double), hipMemcpyDeviceToHost, st), "download H1");
  AFQMC_HIP(hipStreamSynchronize(st), "set-up synchronise");
  double l2 = 0.0;
  for (double v : hl) l2 += v * v;
  s.const_c = s.ecore - 0.5 * l2;
  double n1 = 0.0;
  for (size_t qq = 0; qq < M; ++qq) {
    double col = 0.0;
    for (size_t pp = 0; pp < M; ++pp) col += std::fabs(hH1[pp * M + qq]);
    n1 = std::max(n1, col);
  }
  {
    afqmc_status r = device_expm(tmp, H1, -0.5 * s.dt, n1, s.M, s.B1, st);
    if (r != AFQMC_OK) return r;
  }
  // trial energy E_HF: the local energy of the walker phi = Psi
  {
    double2 *phi_t = nullptr, *e_t = nullptr;
    if (!tmp.get(&phi_t, M * Nt) || !tmp.get(&e_t, 3))
      return fail(AFQMC_ERR_OOM, "device allocation failed (trial energy)");
    std::vector<double2> hphi(M * Nt);
    for (size_t k = 0; k < M * Nt; ++k) hphi[k] = make_double2(d.trial[k], 0.0);
    AFQMC_HIP(hipMemcpyAsync(phi_t, hphi.data(), M * Nt * sizeof(double2), hipMemcpyHostToDevice, st),
              "upload trial walker");
    const int prec = s.precision;
    s.precision = AFQMC_FP64;  // the trial energy (and default E_T) in FP64
    afqmc_status r = local_energy_sys(nullptr, s, phi_t, 1, e_t, nullptr, nullptr, st);
    s.precision = prec;
    if (r != AFQMC_OK) return r;
    double2 he[3];
    AFQMC_HIP(hipMemcpyAsync(he, e_t, sizeof(he), hipMemcpyDeviceToHost, st), "download trial energy");
    AFQMC_HIP(hipStreamSynchronize(st), "set-up synchronise");
    s.e_hf = he[0].x;
  }
  s.ex_mode = c->opt.ex_mode;  // the trial energy above used the full exchange
  return AFQMC_OK;
}

// Set-up tuner.  Launch shapes are timed on the system's own sizes, with the
// operands filled by a fixed pattern:
//  * the exchange kernels: the walker tiling of the FP64 kernel (1, 2 or 4
//    walkers per workgroup; the four waves then split 4, 2 or 1 ways over
//    Cholesky vectors) and the tile order (tile_of: Cholesky block fastest, or
//    groups of 4, 8 or 16 walker blocks);
//  * the V_HS product: kVhsShapes workgroup tiles;
//  * the Taylor-term kernel: its row tiles (48 or 32 rows; 48, 32 or 64 for
//    FP32 propagation).
// Every choice changes speed only: each kernel sums the same terms in the same
// order whatever the shape.  Choices are kept per problem shape (M, N_alpha,
// N_beta, G, W, precision, propagation precision) for the rest of the process,
// so every context of one shape launches alike, and, with options.tune_cache,
// in a file of JSON lines that later processes read instead of timing.
struct TuneKey {
  std::array<int, 7> k;
  bool operator<(const TuneKey &o) const { return k < o.k; }
};
struct TuneChoice {
  int ex_tile = -1, ex_order = -1, vhs = -1, taylor = -1;   // -1: not tuned
};
const char *const kTuneNames[7] = {"M", "Na", "Nb", "G", "W", "precision", "prop32"};

// integer value of "name": in one JSON line (false if absent or malformed)
bool json_int(const std::string &line, const char *name, int *out) {
  const std::string pat = std::string("\"") + name + "\"";
  size_t p = line.find(pat);
  if (p == std::string::npos) return false;
  p = line.find(':', p + pat.size());
  if (p == std::string::npos) return false;
  ++p;
  while (p < line.size() && (line[p] == ' ' || line[p] == '\t')) ++p;
  char *end = nullptr;
  const long v = strtol(line.c_str() + p, &end, 10);
  if (end == line.c_str() + p) return false;
  *out = (int)v;
  return true;
}

// the last line of the cache file for `key` (parts absent in it stay -1)
void cache_read(const std::string &path, const TuneKey &key, TuneChoice *ch) {
  FILE *f = fopen(path.c_str(), "r");
  if (!f) return;
  char buf[1024];
  while (fgets(buf, sizeof buf, f)) {
    const std::string line(buf);
    bool match = true;
    for (int i = 0; i < 7 && match; ++i) {
      int v;
      match = json_int(line, kTuneNames[i], &v) && v == key.k[i];
    }
    if (!match) continue;
    TuneChoice c;
    (void)json_int(line, "ex_tile", &c.ex_tile);
    (void)json_int(line, "ex_order", &c.ex_order);
    (void)json_int(line, "vhs_tile", &c.vhs);
    (void)json_int(line, "taylor_tile", &c.taylor);
    *ch = c;
  }
  fclose(f);
}

bool cache_append(const std::string &path, const TuneKey &key, const TuneChoice &c) {
  FILE *f = fopen(path.c_str(), "a");
  if (!f) return false;
  std::string line = "{";
  for (int i = 0; i < 7; ++i) line += std::string("\"") + kTuneNames[i] + "\": " + std::to_string(key.k[i]) + ", ";
  line += "\"ex_tile\": " + std::to_string(c.ex_tile) + ", \"ex_order\": " + std::to_string(c.ex_order) +
          ", \"vhs_tile\": " + std::to_string(c.vhs) + ", \"taylor_tile\": " + std::to_string(c.taylor) + "}\n";
  const bool ok = fputs(line.c_str(), f) >= 0;
  return fclose(f) == 0 && ok;
}

// median-free timing: one warm-up call, then two timed calls between events
template <class F>
hipError_t time_ms(F run, hipStream_t st, hipEvent_t e0, hipEvent_t e1, float *ms) {
  hipError_t e = run();
  if (e != hipSuccess) return e;
  if ((e = hipEventRecord(e0, st)) != hipSuccess) return e;
  for (int r = 0; r < 2; ++r)
    if ((e = run()) != hipSuccess) return e;
  if ((e = hipEventRecord(e1, st)) != hipSuccess) return e;
  if ((e = hipEventSynchronize(e1)) != hipSuccess) return e;
  return hipEventElapsedTime(ms, e0, e1);
}

hipError_t tune_exchange_shape(System &s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, TuneChoice *ch) {
  const bool lp = s.precision != AFQMC_FP64;
  hipError_t err = launch_fill_pattern2(s.theta, (long)s.W * s.M * s.Nt, st);
  if (lp)
    for (int sp = 0; sp < 2 && err == hipSuccess; ++sp) err = lp_prepare_rhs(s, s.theta, s.W, sp, st);
  if (err != hipSuccess) return err;
  auto run = [&]() -> hipError_t {
    for (int sp = 0; sp < 2; ++sp) {
      hipError_t e = lp ? launch_exchange_lp(s, s.W, sp, st, s.fbpart) : launch_exchange(s, s.theta, s.W, st, s.fbpart, sp);
      if (e != hipSuccess) return e;
    }
    return hipSuccess;
  };
  float best_ms = 0.0f;
  for (int wx : {1, 2, 4}) {
    if (lp && wx != 2) continue;  // the reduced-precision kernels have a fixed walker tiling
    const ExchangePlan p0 = exchange_plan(s.Na, s.G, wx), p1 = exchange_plan(s.Nb, s.G, wx);
    if ((s.Na > 0 && !p0.mfma) || (s.Nb > 0 && !p1.mfma)) continue;
    s.ex_plan[0] = p0;
    s.ex_plan[1] = p1;
    if ((err = exchange_enable_lds(s)) != hipSuccess) return err;
    for (int group : {0, 4, 8, 16}) {
      s.ex_group = group;
      float ms = 0.0f;
      if ((err = time_ms(run, st, e0, e1, &ms)) != hipSuccess) return err;
      if (ch->ex_tile < 0 || ms < best_ms) {
        ch->ex_tile = wx;
        ch->ex_order = group;
        best_ms = ms;
      }
    }
  }
  return hipSuccess;
}

constexpr int kTuneRounds = 3;   // interleaved timing rounds per candidate (the best counts)

hipError_t tune_vhs_shape(System &s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, TuneChoice *ch) {
  hipError_t err = launch_fill_pattern2(reinterpret_cast<double2 *>(s.yp), (long)s.W * s.G, st);
  if (err != hipSuccess) return err;
  // the shapes lie within a few per cent of each other: each keeps its best of
  // kTuneRounds interleaved timings
  float best[kVhsShapes];
  for (int r = 0; r < kTuneRounds; ++r)
    for (int v = 0; v < kVhsShapes; ++v) {
      s.vhs_shape = v;
      float ms = 0.0f;
      if ((err = time_ms([&]() { return launch_vhs(s, s.W, st, false); }, st, e0, e1, &ms)) != hipSuccess) return err;
      if (r == 0 || ms < best[v]) best[v] = ms;
    }
  for (int v = 0; v < kVhsShapes; ++v)
    if (ch->vhs < 0 || best[v] < best[ch->vhs]) ch->vhs = v;
  return hipSuccess;
}

hipError_t tune_taylor_shape(System &s, hipStream_t st, hipEvent_t e0, hipEvent_t e1, TuneChoice *ch) {
  // V_HS from pattern fields, then one term from a pattern walker slab
  hipError_t err = launch_fill_pattern2(reinterpret_cast<double2 *>(s.yp), (long)s.W * s.G, st);
  if (err == hipSuccess) err = launch_vhs(s, s.W, st, false);
  if (err == hipSuccess) err = launch_fill_pattern2(s.tA, (long)s.W * s.M * s.Nt, st);
  if (err == hipSuccess && s.prop32) err = launch_c128_to_c64(s.tA, (long)s.W * s.M * s.Nt, s.tA32, st);
  if (err != hipSuccess) return err;
  const int nshape = taylor_shapes(s);
  float best[8];
  for (int r = 0; r < kTuneRounds; ++r)
    for (int v = 0; v < nshape; ++v) {
      s.taylor_shape = v;
      auto run = [&]() {
        return s.prop32 ? launch_taylor_f32(s, s.tA32, s.tB32, 1.0, s.W, st, 0)
                        : launch_taylor_term(s, s.tA, s.tB, 1.0, s.W, st, 0);
      };
      float ms = 0.0f;
      if ((err = time_ms(run, st, e0, e1, &ms)) != hipSuccess) return err;
      if (r == 0 || ms < best[v]) best[v] = ms;
    }
  for (int v = 0; v < nshape; ++v)
    if (ch->taylor < 0 || best[v] < best[ch->taylor]) ch->taylor = v;
  return hipSuccess;
}

afqmc_status tune_system(afqmc_ctx *c, System &s, hipStream_t st) {
  static std::mutex mu;
  static std::map<TuneKey, TuneChoice> chosen;
  const TuneKey key{{s.M, s.Na, s.Nb, s.G, s.W, s.precision, s.prop32 ? 1 : 0}};
  if (c->taylor_fixed >= taylor_shapes(s)) return fail(AFQMC_ERR_ARG, "reserved[4]: no such Taylor tile shape");
  // which parts this context leaves to the tuner
  const bool want_ex = c->tune && !c->ex_wx_forced && s.ex_mfma;
  const bool want_vhs = c->tune && c->vhs_fixed < 0 && s.use_mfma_gemm && s.Lp && !s.prop32;
  const bool want_taylor = c->tune && c->taylor_fixed < 0 && (s.prop32 || taylor_walker_split(s));
  TuneChoice ch;
  {
    std::lock_guard<std::mutex> lock(mu);
    auto it = chosen.find(key);
    if (it != chosen.end()) ch = it->second;
  }
  const bool from_file = !c->tune_cache.empty() &&
                         ((want_ex && ch.ex_tile < 0) || (want_vhs && ch.vhs < 0) || (want_taylor && ch.taylor < 0));
  if (from_file) {
    TuneChoice f;
    cache_read(c->tune_cache, key, &f);
    if (ch.ex_tile < 0) { ch.ex_tile = f.ex_tile; ch.ex_order = f.ex_order; }
    if (ch.vhs < 0) ch.vhs = f.vhs;
    if (ch.taylor < 0) ch.taylor = f.taylor;
  }
  const bool time_ex = want_ex && ch.ex_tile < 0, time_vhs = want_vhs && ch.vhs < 0,
             time_taylor = want_taylor && ch.taylor < 0;
  if (time_ex || time_vhs || time_taylor) {
    hipEvent_t e0, e1;
    AFQMC_HIP(hipEventCreate(&e0), "event create");
    if (hipEventCreate(&e1) != hipSuccess) {
      (void)hipEventDestroy(e0);
      return fail(AFQMC_ERR_HIP, "event create");
    }
    hipError_t err = hipSuccess;
    if (time_ex) err = tune_exchange_shape(s, st, e0, e1, &ch);
    if (err == hipSuccess && time_vhs) err = tune_vhs_shape(s, st, e0, e1, &ch);
    if (err == hipSuccess && time_taylor) err = tune_taylor_shape(s, st, e0, e1, &ch);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (err != hipSuccess) return fail(AFQMC_ERR_HIP, std::string("launch-shape tuning: ") + hipGetErrorString(err));
    s.cache_phi = nullptr;  // Theta and the walker slabs hold tuning patterns
    if (!c->tune_cache.empty() && !cache_append(c->tune_cache, key, ch))
      return fail(AFQMC_ERR_ARG, "cannot write the tuning cache " + c->tune_cache);
  }
  {
    std::lock_guard<std::mutex> lock(mu);
    TuneChoice &kept = chosen[key];
    if (ch.ex_tile >= 0) { kept.ex_tile = ch.ex_tile; kept.ex_order = ch.ex_order; }
    if (ch.vhs >= 0) kept.vhs = ch.vhs;
    if (ch.taylor >= 0) kept.taylor = ch.taylor;
  }
  if (want_ex && ch.ex_tile > 0) {
    s.ex_plan[0] = exchange_plan(s.Na, s.G, ch.ex_tile);
    s.ex_plan[1] = exchange_plan(s.Nb, s.G, ch.ex_tile);
    s.ex_group = ch.ex_order;
  }
  if (s.ex_mfma) AFQMC_HIP(exchange_enable_lds(s), "exchange kernel LDS attribute");
  s.vhs_shape = c->vhs_fixed >= 0 ? c->vhs_fixed : (want_vhs && ch.vhs >= 0 ? ch.vhs : 0);
  s.taylor_shape = c->taylor_fixed >= 0 ? c->taylor_fixed : (want_taylor && ch.taylor >= 0 ? ch.taylor : 0);
  return AFQMC_OK;
}

// Estimated cost of one step of system s (flops; for spreading systems over lanes).
double step_cost(const System &s) {
  const double M = s.M, G = s.G, n2 = (double)s.Na * s.Na + (double)s.Nb * s.Nb;
  return s.W * (4.0 * n2 * M * G + 4.0 * G * M * M + 64.0 * M * M * s.Nt) + 2.0e7;
}

// Runs body(i, stream) for every system: in order on the caller's stream, or
// spread over the context's lanes, forked after the work already enqueued on
// `st` and joined back into it.  Each system's work stays in order on its lane.
template <class F>
afqmc_status for_each_system(afqmc_ctx *c, hipStream_t st, F body) {
  const int n = (int)c->sys.size();
  if (c->lanes.empty()) {
    for (int i = 0; i < n; ++i) {
      afqmc_status r = body(i, st);
      if (r != AFQMC_OK) return r;
    }
    return AFQMC_OK;
  }
  AFQMC_HIP(hipEventRecord(c->fork_ev, st), "event record");
  for (hipStream_t l : c->lanes) AFQMC_HIP(hipStreamWaitEvent(l, c->fork_ev, 0), "stream wait");
  afqmc_status res = AFQMC_OK;
  for (int i = 0; i < n && res == AFQMC_OK; ++i) res = body(i, c->lanes[c->lane_of[i]]);
  // join every lane, also after a failure, so that no lane runs ahead of `st`
  for (size_t l = 0; l < c->lanes.size(); ++l) {
    AFQMC_HIP(hipEventRecord(c->join_ev[l], c->lanes[l]), "event record");
    AFQMC_HIP(hipStreamWaitEvent(st, c->join_ev[l], 0), "stream wait");
  }
  return res;
}

// Internal streams of a system set, with systems assigned largest first to the
// least-loaded lane.
afqmc_status make_lanes(afqmc_ctx *c, int nl) {
  const int n = (int)c->sys.size();
  if (nl <= 1 || n <= 1) return AFQMC_OK;
  nl = std::min(nl, n);
  for (int l = 0; l < nl; ++l) {
    hipStream_t h;
    AFQMC_HIP(hipStreamCreateWithFlags(&h, hipStreamNonBlocking), "stream create");
    c->lanes.push_back(h);
    hipEvent_t e;
    AFQMC_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event create");
    c->join_ev.push_back(e);
  }
  AFQMC_HIP(hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming), "event create");
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(),
                   [&](int a, int b) { return step_cost(c->sys[a]) > step_cost(c->sys[b]); });
  std::vector<double> load(nl, 0.0);
  c->lane_of.assign(n, 0);
  for (int i : order) {
    const int l = (int)(std::min_element(load.begin(), load.end()) - load.begin());
    c->lane_of[i] = l;
    load[l] += step_cost(c->sys[i]);
  }
  return AFQMC_OK;
}

}  // namespace

extern "C" {

afqmc_status afqmc_default_options(afqmc_options *opt) {
  if (!opt) return fail(AFQMC_ERR_ARG, "opt is NULL");
  memset(opt, 0, sizeof(*opt));
  opt->precision = AFQMC_FP64;
  opt->taylor_order = 6;
  opt->fb_cap = 1.0;
  opt->e_shift = NAN;
  opt->mem_limit_bytes = 0;
  opt->streams = 0;
  opt->use_graph = 0;
  opt->tune = 1;
  opt->ex_mode = AFQMC_EX_FULL;
  opt->cv_fraction = 0.125;
  opt->cv_seed = 7;
  opt->deterministic = 1;
  return AFQMC_OK;
}

const char *afqmc_last_error(void) { return g_last_error.c_str(); }

afqmc_status afqmc_setup_hamiltonian(const afqmc_system_desc *sys, int32_t nsys, const afqmc_options *opt,
                                     void *hip_stream, afqmc_ctx **out) {
  if (!out) return fail(AFQMC_ERR_ARG, "out is NULL");
  *out = nullptr;
  if (!sys || nsys <= 0) return fail(AFQMC_ERR_ARG, "need nsys >= 1 system descriptions");
  afqmc_options o;
  if (opt) o = *opt;
  else afqmc_default_options(&o);
  if (o.precision != AFQMC_FP64 && o.precision != AFQMC_FP32_CONTRACT && o.precision != AFQMC_BF16X3_CONTRACT &&
      o.precision != AFQMC_BF16X2_CONTRACT && o.precision != AFQMC_FP16_TSPLIT_CONTRACT &&
      o.precision != AFQMC_BF16_TSPLIT_CONTRACT)
    return fail(AFQMC_ERR_ARG, "unknown precision");
  if (o.taylor_order < 1 || o.taylor_order > 16) return fail(AFQMC_ERR_ARG, "taylor_order must be in 1..16");
  if (std::isnan(o.fb_cap) || std::isinf(o.fb_cap)) return fail(AFQMC_ERR_ARG, "fb_cap must be finite");
  if (o.streams < 0) return fail(AFQMC_ERR_ARG, "streams must be >= 0");
  if (o.prop_precision != AFQMC_FP64 && o.prop_precision != AFQMC_FP32_CONTRACT)
    return fail(AFQMC_ERR_ARG, "prop_precision must be AFQMC_FP64 or AFQMC_FP32_CONTRACT");
  if (o.ex_mode != AFQMC_EX_FULL && o.ex_mode != AFQMC_EX_CV) return fail(AFQMC_ERR_ARG, "unknown ex_mode");
  if (!(o.cv_fraction > 0.0 && o.cv_fraction <= 1.0)) return fail(AFQMC_ERR_ARG, "cv_fraction must be in (0, 1]");
  if (o.deterministic != 1)
    return fail(AFQMC_ERR_ARG, "deterministic must be 1: only fixed-order reductions are provided");
  if (o.ex_mode == AFQMC_EX_CV)
    for (int i = 0; i < nsys; ++i)
      if (sys[i].nwalkers > kCvMaxWalkers)
        return fail(AFQMC_ERR_UNSUPPORTED, "the control-variate exchange supports at most " +
                                               std::to_string(kCvMaxWalkers) + " walkers per system");
  for (int i = 0; i < nsys; ++i) {
    std::string why;
    if (!valid_desc(sys[i], why)) return fail(AFQMC_ERR_ARG, "system " + std::to_string(i) + ": " + why);
  }
  for (int i = 0; i < nsys; ++i)
    if (std::max(sys[i].nalpha, sys[i].nbeta) > kMaxSpinOrbitals)
      return fail(AFQMC_ERR_UNSUPPORTED, "system " + std::to_string(i) + ": a spin block wider than " +
                                             std::to_string(kMaxSpinOrbitals) + " orbitals is not supported");
  afqmc_ctx *c = new (std::nothrow) afqmc_ctx();
  if (!c) return fail(AFQMC_ERR_OOM, "host allocation failed");
  c->opt.precision = o.precision;
  if (o.precision != AFQMC_FP64 && (o.reserved[0] & 1))
    { delete c; return fail(AFQMC_ERR_UNSUPPORTED, "reduced precision needs the MFMA exchange kernel"); }
  c->opt.taylor_order = o.taylor_order;
  c->opt.fb_cap = o.fb_cap;
  c->opt.ex_mode = o.ex_mode;
  c->opt.cv_fraction = o.cv_fraction;
  c->opt.cv_seed = o.cv_seed;
  c->opt.prop_precision = o.prop_precision;
  c->force_valu_exchange = (o.reserved[0] & 1) != 0;
  c->force_valu_gemm = (o.reserved[0] & 2) != 0;
  c->debug_bits = o.reserved[0];
  if (o.reserved[3] >= 1 && o.reserved[3] <= kVhsShapes) c->vhs_fixed = o.reserved[3] - 1;
  if (o.reserved[4] >= 1 && o.reserved[4] <= 4) c->taylor_fixed = o.reserved[4] - 1;
  if (o.tune_cache) c->tune_cache = o.tune_cache;
  if (o.reserved[1] == 1 || o.reserved[1] == 2 || o.reserved[1] == 4) {
    c->ex_wx = o.reserved[1];
    c->ex_wx_forced = true;
  }
  if (o.reserved[2] > 0) {
    c->ex_group = o.reserved[2] == 1 ? 0 : o.reserved[2];
    c->ex_wx_forced = true;
  }
  c->tune = o.tune != 0;
  c->use_graph = o.use_graph != 0;
  (void)hipGetDevice(&c->device);
  {
    afqmc_status r = bind_scratch(c->device);
    if (r != AFQMC_OK) {
      delete c;
      return r;
    }
  }
  c->sys.resize(nsys);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  uint64_t used = 0;
  for (int i = 0; i < nsys; ++i) {
    afqmc_status r = setup_one(c, sys[i], c->sys[i], st, &used, o.mem_limit_bytes);
    System &sy = c->sys[i];
    if (r == AFQMC_OK) r = tune_system(c, sy, st);
    if (r == AFQMC_OK && sy.Lp && sy.L) {
      // after set-up only the packed triangles are read: give the full tensor back
      if (hipStreamSynchronize(st) != hipSuccess) r = fail(AFQMC_ERR_HIP, "set-up failed on the device");
      else {
        free_one(c, sy.L);
        sy.L = nullptr;
        sy.bytes -= 8ull * sy.G * sy.M * sy.M;
        if (sy.Lp32) {
          // FP32 propagation reads only the FP32 copy
          free_one(c, sy.Lp);
          sy.Lp = nullptr;
          sy.bytes -= 4ull * sy.G * sy.M * (sy.M + 1);
        }
      }
    }
    if (r != AFQMC_OK) {
      (void)hipStreamSynchronize(st);
      release(c);
      delete c;
      return r;
    }
    sy.e_shift = std::isnan(o.e_shift) ? sy.e_hf : o.e_shift;
    if (launch_set_e_shift(sy, sy.e_shift, st) != hipSuccess) {
      (void)hipStreamSynchronize(st);
      release(c);
      delete c;
      return fail(AFQMC_ERR_HIP, "energy-shift kernel");
    }
  }
  afqmc_status r = make_lanes(c, o.streams == 0 ? 4 : o.streams);
  for (System &sy : c->sys) {
    if (r != AFQMC_OK || !taylor_walker_split(sy) || sy.W < 2) continue;
    if (hipStreamCreateWithFlags(&sy.half_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&sy.half_fork, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&sy.half_join, hipEventDisableTiming) != hipSuccess)
      r = fail(AFQMC_ERR_HIP, "Taylor stream or event create");
  }
  if (r == AFQMC_OK && c->use_graph) {
    if (hipStreamCreateWithFlags(&c->cap_stream, hipStreamNonBlocking) != hipSuccess ||
        hipEventCreateWithFlags(&c->g_in, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&c->g_out, hipEventDisableTiming) != hipSuccess)
      r = fail(AFQMC_ERR_HIP, "graph stream or event create");
  }
  if (r == AFQMC_OK && hipStreamSynchronize(st) != hipSuccess) r = fail(AFQMC_ERR_HIP, "set-up failed on the device");
  if (r != AFQMC_OK) {
    release(c);
    delete c;
    return r;
  }
  *out = c;
  return AFQMC_OK;
}

// phi <- B1 T(sqrt(dt) V_HS) B1 phi from the rows already in s.yp, then the
// overlap pass of the new walkers (log-overlaps into s.logo_new, Theta into
// s.theta with `want_theta`).  `imag` says V_HS is purely imaginary (free
// projection): only its imaginary plane is formed and contracted where the
// Taylor kernels allow it.
static afqmc_status apply_propagator(afqmc_ctx *ctx, System &s, double2 *phi, bool want_theta, bool imag,
                                     hipStream_t st) {
  const int W = s.W;
  const bool half = imag && free_half_supported(s);
  const int kbeg = half ? s.M : 0;
  {
    Phase ph(ctx, AFQMC_PH_VHS, st);
    AFQMC_HIP(launch_vhs(s, W, st, half), "V_HS kernel");
  }
  // The dedicated FP64 kernel takes the first term straight from tacc = B1 phi
  // without adding to it, and the second term adds its input and output, so
  // the series needs no copy of B1 phi.
  const bool fold = !s.prop32 && taylor_walker_split(s) && ctx->opt.taylor_order >= 2;
  {
    Phase ph(ctx, AFQMC_PH_ONE_BODY, st);
    AFQMC_HIP(launch_b1(s, phi, s.tacc, W, st), "one-body kernel");
    if (!s.prop32 && !fold)
      AFQMC_HIP(hipMemcpyAsync(s.tA, s.tacc, (size_t)W * s.M * s.Nt * sizeof(double2), hipMemcpyDeviceToDevice, st),
                "copy");
  }
  {
    Phase ph(ctx, AFQMC_PH_TAYLOR, st);
    if (s.prop32) {
      // terms in FP32 from an FP32 copy of B1 phi; the series accumulates in FP64 (tacc)
      AFQMC_HIP(launch_c128_to_c64(s.tacc, (long)W * s.M * s.Nt, s.tA32, st), "conversion kernel");
      float2 *tin = s.tA32, *tout = s.tB32;
      for (int n = 1; n <= ctx->opt.taylor_order; ++n) {
        AFQMC_HIP(launch_taylor_f32(s, tin, tout, 1.0 / n, W, st, kbeg), "FP32 Taylor kernel");
        std::swap(tin, tout);
      }
    } else {
      // with a second stream, walkers [W1, W) take their terms there: the
      // launch tail of each term of one half overlaps the other half's work
      // (not while a graph is being recorded: recording it crashed the host runtime)
      const bool split = s.half_stream != nullptr && W >= 2 && !ctx->capturing;
      const int W1 = split ? (W + 1) / 2 : W;
      if (split) {
        AFQMC_HIP(hipEventRecord(s.half_fork, st), "event record");
        AFQMC_HIP(hipStreamWaitEvent(s.half_stream, s.half_fork, 0), "stream wait");
      }
      double2 *tin = fold ? s.tacc : s.tA, *tout = fold ? s.tA : s.tB;
      hipError_t e = hipSuccess;
      for (int n = 1; n <= ctx->opt.taylor_order && e == hipSuccess; ++n) {
        const int acc = !fold ? 1 : n == 1 ? 0 : n == 2 ? 2 : 1;
        if (split) {
          e = launch_taylor_mfma(s, tin, tout, 1.0 / n, W1, st, kbeg, 0, acc);
          if (e == hipSuccess) e = launch_taylor_mfma(s, tin, tout, 1.0 / n, W - W1, s.half_stream, kbeg, W1, acc);
        } else if (fold) {
          e = launch_taylor_mfma(s, tin, tout, 1.0 / n, W, st, kbeg, 0, acc);
        } else {
          e = launch_taylor_term(s, tin, tout, 1.0 / n, W, st, kbeg);
        }
        if (fold && n == 1) {
          tin = s.tA;
          tout = s.tB;
        } else {
          std::swap(tin, tout);
        }
      }
      if (split) {  // joined also after a failure, so that the second stream never runs ahead of `st`
        AFQMC_HIP(hipEventRecord(s.half_join, s.half_stream), "event record");
        AFQMC_HIP(hipStreamWaitEvent(st, s.half_join, 0), "stream wait");
      }
      AFQMC_HIP(e, "Taylor kernel");
    }
  }
  {
    Phase ph(ctx, AFQMC_PH_ONE_BODY, st);
    AFQMC_HIP(launch_b1(s, s.tacc, phi, W, st), "one-body kernel");
  }
  {
    Phase ph(ctx, AFQMC_PH_OVERLAP, st);
    AFQMC_HIP(launch_ovlp_theta(phi, s.trial, s.M, s.Na, s.Nb, W, want_theta ? s.theta : nullptr, s.logo_new,
                                s.stat_new, nullptr, st, s.opart, s.ospart),
              "overlap kernel");
  }
  return AFQMC_OK;
}

// One propagation step of system s.  With `reuse`, theta / fbpart already hold
// Theta and the vbias partials of the current walkers, and their log-overlaps
// are taken from walkers.log_ovlp.  With `want_theta` the overlap pass after
// the step also writes Theta of the new walkers (for a local energy next).
static afqmc_status propagate_sys(afqmc_ctx *ctx, System &s, const afqmc_walkers &wk, const double *x, bool reuse,
                                  bool want_theta, hipStream_t st, bool ready = false) {
  double2 *phi = static_cast<double2 *>(wk.phi);
  const int W = s.W;
  if (ready) {
    // Theta, log-overlaps, singular markers and vbias partials already computed
  } else if (reuse) {
    AFQMC_HIP(hipMemcpyAsync(s.logo_now, wk.log_ovlp, (size_t)W * sizeof(double2), hipMemcpyDeviceToDevice, st),
              "copy");
    AFQMC_HIP(hipMemcpyAsync(s.stat_now, s.stat_new, (size_t)W * sizeof(uint32_t), hipMemcpyDeviceToDevice, st),
              "copy");
  } else {
    {
      Phase ph(ctx, AFQMC_PH_OVERLAP, st);
      AFQMC_HIP(launch_ovlp_theta(phi, s.trial, s.M, s.Na, s.Nb, W, s.theta, s.logo_now, s.stat_now, nullptr, st, s.opart, s.ospart),
                "overlap kernel");
    }
    {
      Phase ph(ctx, AFQMC_PH_FORCE_BIAS, st);
      AFQMC_HIP(launch_force_bias_gemm(s, s.theta, W, st), "force-bias kernel");
    }
    s.fb_slices = s.fb_ksplit;
  }
  {
    Phase ph(ctx, AFQMC_PH_FB_EPILOGUE, st);
    AFQMC_HIP(launch_fb_propagate_epilogue(s, ctx->opt, x, W, wk.flags, s.fb_slices, st), "force-bias epilogue");
  }
  afqmc_status r = apply_propagator(ctx, s, phi, want_theta, false, st);
  if (r != AFQMC_OK) return r;
  {
    Phase ph(ctx, AFQMC_PH_WEIGHT, st);
    AFQMC_HIP(launch_weight_update(s, wk, W, st), "weight kernel");
  }
  return AFQMC_OK;
}

// One free-projection step of system s (fields, propagator, amplitude update).
static afqmc_status free_propagate_sys(afqmc_ctx *ctx, System &s, const afqmc_walkers &wk, const double *x,
                                       double2 *amp, bool want_theta, hipStream_t st) {
  {
    Phase ph(ctx, AFQMC_PH_FB_EPILOGUE, st);
    AFQMC_HIP(launch_free_fields(s, x, s.W, wk.flags, st), "field kernel");
  }
  afqmc_status r = apply_propagator(ctx, s, static_cast<double2 *>(wk.phi), want_theta, true, st);
  if (r != AFQMC_OK) return r;
  {
    Phase ph(ctx, AFQMC_PH_WEIGHT, st);
    AFQMC_HIP(launch_free_amplitude(s, wk, amp, s.W, st), "amplitude kernel");
  }
  return AFQMC_OK;
}

static void invalidate_caches(afqmc_ctx *ctx) {
  for (System &s : ctx->sys) s.cache_phi = nullptr;
}

static afqmc_status check_walkers(const afqmc_walkers &w, int i) {
  if (!w.phi || !w.weight || !w.log_ovlp || !w.flags)
    return fail(AFQMC_ERR_ARG, "walkers of system " + std::to_string(i) + " have a NULL buffer");
  return AFQMC_OK;
}

afqmc_status afqmc_propagate(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *hip_stream) {
  if (!ctx || !w || !x) return fail(AFQMC_ERR_ARG, "NULL context, walkers or fields");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!x[i]) return fail(AFQMC_ERR_ARG, "fields of system " + std::to_string(i) + " are NULL");
  }
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    return propagate_sys(ctx, ctx->sys[i], w[i], x[i], false, false, ls);
  });
}

}  // extern "C"

namespace {

// One walker step of system i on stream ls (arguments already checked):
// propagation, optional re-orthogonalisation, local energy and estimator
// record (est may be NULL).
afqmc_status step_one(afqmc_ctx *ctx, int i, const afqmc_walkers &wk, const double *x, void *e_out, double *est,
                      uint32_t flags, hipStream_t ls) {
  System &s = ctx->sys[i];
  const bool reuse = !(flags & AFQMC_STEP_FRESH) && s.cache_phi == wk.phi;
  s.cache_phi = nullptr;
  bool ready = false;
  if (!reuse && s.ex_mfma && s.ex_mode == AFQMC_EX_FULL) {
    // a fresh start takes vbias by the route every later step takes (the
    // trace of the exchange matrices), so a run restarted from its walker
    // state repeats the uninterrupted run bit for bit
    {
      Phase ph(ctx, AFQMC_PH_OVERLAP, ls);
      AFQMC_HIP(launch_ovlp_theta(static_cast<const double2 *>(wk.phi), s.trial, s.M, s.Na, s.Nb, s.W, s.theta,
                                  s.logo_now, s.stat_now, nullptr, ls, s.opart, s.ospart),
                "overlap kernel");
    }
    afqmc_status r = exchange_sys(ctx, s, s.theta, s.W, s.fbpart, ls);
    if (r != AFQMC_OK) return r;
    s.fb_slices = 2;
    ready = true;
  }
  afqmc_status r = propagate_sys(ctx, s, wk, x, reuse, true, ls, ready);
  if (r != AFQMC_OK) return r;
  if (flags & AFQMC_STEP_REORTHO) {
    Phase ph(ctx, AFQMC_PH_REORTHO, ls);
    AFQMC_HIP(launch_mgs(static_cast<double2 *>(wk.phi), s.M, s.Na, s.Nb, s.W, static_cast<double2 *>(wk.log_ovlp),
                         ls, reinterpret_cast<double *>(s.opart)),
              "Gram-Schmidt kernel");
  }
  r = local_energy_sys(ctx, s, static_cast<const double2 *>(wk.phi), s.W, static_cast<double2 *>(e_out), est,
                       wk.weight, ls, true);
  if (r != AFQMC_OK) return r;
  s.cache_phi = wk.phi;
  return AFQMC_OK;
}

// The body of afqmc_step (arguments already checked).
afqmc_status step_body(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *e_out,
                       double *est_out, uint32_t flags, hipStream_t st) {
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    return step_one(ctx, i, w[i], x[i], e_out[i], est_out ? est_out + 4 * i : nullptr, flags, ls);
  });
}

// Arguments of one block of afqmc_run_block.
struct BlockArgs {
  const afqmc_walkers *w;
  const double *const *x;
  int nsteps;
  int64_t step0;
  int reortho_every;
  void *const *e_out;
  double *const *est;
  const double *const *u;
  uint32_t flags;
};

// The body of afqmc_run_block: every system runs its whole block on its lane.
afqmc_status block_body(afqmc_ctx *ctx, const BlockArgs &b, hipStream_t st) {
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    const size_t per_step = (size_t)s.W * s.G;
    for (int k = 0; k < b.nsteps; ++k) {
      uint32_t f = (k == 0) ? (b.flags & AFQMC_STEP_FRESH) : 0u;
      if (b.reortho_every > 0 && (b.step0 + k + 1) % b.reortho_every == 0) f |= AFQMC_STEP_REORTHO;
      afqmc_status r = step_one(ctx, i, b.w[i], b.x[i] + (size_t)k * per_step, b.e_out[i],
                                b.est[i] + (size_t)4 * k, f, ls);
      if (r != AFQMC_OK) return r;
    }
    if (b.u) {
      s.cache_phi = nullptr;
      AFQMC_HIP(launch_comb(s, b.w[i].weight, static_cast<double2 *>(b.w[i].phi),
                            static_cast<double2 *>(b.w[i].log_ovlp), b.w[i].flags, b.u[i], nullptr, ls),
                "population control kernels");
    }
    if (b.flags & AFQMC_BLOCK_FEEDBACK) AFQMC_HIP(launch_block_e_shift(s, b.est[i], b.nsteps, ls), "energy-shift kernel");
    return AFQMC_OK;
  });
}

// Records `body` into a hipGraph on the context's own stream (never the
// caller's, which may be the legacy default stream) the first time `key` is
// seen and replays it after that; `after_replay` restores the host-side state a
// recorded call leaves behind.  Up to eight recordings are kept (a run
// alternates between a few: the first step, plain and re-orthogonalising steps,
// blocks).
template <class Body, class After>
afqmc_status run_graph(afqmc_ctx *ctx, const std::vector<uintptr_t> &key, hipStream_t st, Body body,
                       After after_replay) {
  hipGraphExec_t exec = nullptr;
  for (auto &g : ctx->graphs)
    if (g.key == key) exec = g.exec;
  if (!exec) {
    AFQMC_HIP(hipStreamBeginCapture(ctx->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    ctx->capturing = true;
    afqmc_status r = body(ctx->cap_stream);
    hipGraph_t graph = nullptr;
    hipError_t e = hipStreamEndCapture(ctx->cap_stream, &graph);
    ctx->capturing = false;
    if (r == AFQMC_OK && e != hipSuccess) r = fail(AFQMC_ERR_HIP, std::string("end capture: ") + hipGetErrorString(e));
    if (r == AFQMC_OK) {
      e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
      if (e != hipSuccess) r = fail(AFQMC_ERR_HIP, std::string("graph instantiate: ") + hipGetErrorString(e));
    }
    if (graph) (void)hipGraphDestroy(graph);
    if (r != AFQMC_OK) {
      for (System &s : ctx->sys) s.cache_phi = nullptr;
      return r;
    }
    if (ctx->graphs.size() == 8) {
      (void)hipGraphExecDestroy(ctx->graphs.front().exec);
      ctx->graphs.erase(ctx->graphs.begin());
    }
    ctx->graphs.push_back({key, exec});
    ++ctx->graph_captures;
  } else {
    after_replay();
    ++ctx->graph_replays;
  }
  AFQMC_HIP(hipEventRecord(ctx->g_in, st), "event record");
  AFQMC_HIP(hipStreamWaitEvent(ctx->cap_stream, ctx->g_in, 0), "stream wait");
  AFQMC_HIP(hipGraphLaunch(exec, ctx->cap_stream), "graph launch");
  AFQMC_HIP(hipEventRecord(ctx->g_out, ctx->cap_stream), "event record");
  AFQMC_HIP(hipStreamWaitEvent(st, ctx->g_out, 0), "stream wait");
  return AFQMC_OK;
}

// afqmc_step through a hipGraph, keyed by the flags, every buffer and whether
// the cached Theta / vbias apply.
afqmc_status step_graph(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *e_out,
                        double *est_out, uint32_t flags, hipStream_t st) {
  std::vector<uintptr_t> key;
  key.push_back(0);  // afqmc_step
  key.push_back(flags);
  key.push_back(reinterpret_cast<uintptr_t>(est_out));
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    const System &s = ctx->sys[i];
    const bool reuse = !(flags & AFQMC_STEP_FRESH) && s.cache_phi == w[i].phi;
    for (const void *p : {(const void *)w[i].phi, (const void *)w[i].weight, (const void *)w[i].log_ovlp,
                          (const void *)w[i].flags, (const void *)x[i], (const void *)e_out[i]})
      key.push_back(reinterpret_cast<uintptr_t>(p));
    key.push_back(reuse ? 1u : 0u);
  }
  return run_graph(
      ctx, key, st, [&](hipStream_t cs) { return step_body(ctx, w, x, e_out, est_out, flags, cs); },
      [&]() {
        for (size_t i = 0; i < ctx->sys.size(); ++i) ctx->sys[i].cache_phi = w[i].phi;
      });
}

// afqmc_run_block through a hipGraph; the key also holds the block length and
// which of its steps re-orthogonalise.
afqmc_status block_graph(afqmc_ctx *ctx, const BlockArgs &b, hipStream_t st) {
  std::vector<uintptr_t> key;
  key.push_back(1);  // afqmc_run_block
  key.push_back(b.flags);
  key.push_back((uintptr_t)b.nsteps);
  key.push_back(b.reortho_every > 0 ? (uintptr_t)(b.step0 % b.reortho_every) : 0u);
  key.push_back((uintptr_t)(b.reortho_every > 0 ? b.reortho_every : 0));
  key.push_back(b.u ? 1u : 0u);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    const System &s = ctx->sys[i];
    const bool reuse = !(b.flags & AFQMC_STEP_FRESH) && s.cache_phi == b.w[i].phi;
    for (const void *p : {(const void *)b.w[i].phi, (const void *)b.w[i].weight, (const void *)b.w[i].log_ovlp,
                          (const void *)b.w[i].flags, (const void *)b.x[i], (const void *)b.e_out[i],
                          (const void *)b.est[i], (const void *)(b.u ? b.u[i] : nullptr)})
      key.push_back(reinterpret_cast<uintptr_t>(p));
    key.push_back(reuse ? 1u : 0u);
  }
  return run_graph(
      ctx, key, st, [&](hipStream_t cs) { return block_body(ctx, b, cs); },
      [&]() {
        for (size_t i = 0; i < ctx->sys.size(); ++i) ctx->sys[i].cache_phi = b.u ? nullptr : b.w[i].phi;
      });
}

}  // namespace

extern "C" {

afqmc_status afqmc_step(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *e_out,
                        double *est_out, uint32_t flags, void *hip_stream) {
  if (!ctx || !w || !x || !e_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers, fields or e_out");
  if (flags & ~(uint32_t)(AFQMC_STEP_REORTHO | AFQMC_STEP_FRESH)) return fail(AFQMC_ERR_ARG, "unknown step flags");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!x[i] || !e_out[i]) return fail(AFQMC_ERR_ARG, "NULL fields or e_out of system " + std::to_string(i));
  }
  if (ctx->use_graph) return step_graph(ctx, w, x, e_out, est_out, flags, st);
  return step_body(ctx, w, x, e_out, est_out, flags, st);
}

afqmc_status afqmc_run_block(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, int32_t nsteps,
                             int64_t step0, int32_t reortho_every, void *const *e_out, double *const *est,
                             const double *const *u, uint32_t flags, void *hip_stream) {
  if (!ctx || !w || !x || !e_out || !est) return fail(AFQMC_ERR_ARG, "NULL context, walkers, fields, e_out or est");
  if (nsteps < 1 || step0 < 0 || reortho_every < 0)
    return fail(AFQMC_ERR_ARG, "need nsteps >= 1, step0 >= 0 and reortho_every >= 0");
  if (flags & ~(uint32_t)(AFQMC_STEP_FRESH | AFQMC_BLOCK_FEEDBACK)) return fail(AFQMC_ERR_ARG, "unknown block flags");
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!x[i] || !e_out[i] || !est[i] || (u && !u[i]))
      return fail(AFQMC_ERR_ARG, "NULL fields, e_out, est or offset of system " + std::to_string(i));
  }
  const BlockArgs b{w, x, nsteps, step0, reortho_every, e_out, est, u, flags};
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (ctx->use_graph) return block_graph(ctx, b, st);
  return block_body(ctx, b, st);
}

afqmc_status afqmc_local_energy(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *e_out, double *est_out,
                                void *hip_stream) {
  if (!ctx || !w || !e_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers or e_out");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!e_out[i]) return fail(AFQMC_ERR_ARG, "e_out of system " + std::to_string(i) + " is NULL");
  }
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    return local_energy_sys(ctx, s, static_cast<const double2 *>(w[i].phi), s.W, static_cast<double2 *>(e_out[i]),
                            est_out ? est_out + 4 * i : nullptr, w[i].weight, ls);
  });
}

afqmc_status afqmc_reorthogonalize(afqmc_ctx *ctx, const afqmc_walkers *w, void *hip_stream) {
  if (!ctx || !w) return fail(AFQMC_ERR_ARG, "NULL context or walkers");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
  }
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    Phase ph(ctx, AFQMC_PH_REORTHO, ls);
    AFQMC_HIP(launch_mgs(static_cast<double2 *>(w[i].phi), s.M, s.Na, s.Nb, s.W,
                         static_cast<double2 *>(w[i].log_ovlp), ls, reinterpret_cast<double *>(s.opart)),
              "Gram-Schmidt kernel");
    return AFQMC_OK;
  });
}

afqmc_status afqmc_overlap(afqmc_ctx *ctx, const afqmc_walkers *w, void *hip_stream) {
  if (!ctx || !w) return fail(AFQMC_ERR_ARG, "NULL context or walkers");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
  }
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    AFQMC_HIP(launch_ovlp_theta(static_cast<const double2 *>(w[i].phi), s.trial, s.M, s.Na, s.Nb, s.W, nullptr,
                                static_cast<double2 *>(w[i].log_ovlp), s.stat_new, w[i].flags, ls, s.opart, s.ospart),
              "overlap kernel");
    return AFQMC_OK;
  });
}

afqmc_status afqmc_greens_function(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *theta_out,
                                   void *hip_stream) {
  if (!ctx || !w || !theta_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers or theta_out");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    if (!w[i].phi || !theta_out[i]) return fail(AFQMC_ERR_ARG, "NULL phi or theta_out");
  }
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    System &s = ctx->sys[i];
    AFQMC_HIP(launch_ovlp_theta(static_cast<const double2 *>(w[i].phi), s.trial, s.M, s.Na, s.Nb, s.W,
                                static_cast<double2 *>(theta_out[i]), s.logo_new, s.stat_new, nullptr, st, s.opart, s.ospart),
              "overlap kernel");
  }
  return AFQMC_OK;
}

afqmc_status afqmc_force_bias(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *vbias_out, void *hip_stream) {
  if (!ctx || !w || !vbias_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers or vbias_out");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    if (!w[i].phi || !vbias_out[i]) return fail(AFQMC_ERR_ARG, "NULL phi or vbias_out");
  }
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    System &s = ctx->sys[i];
    AFQMC_HIP(launch_ovlp_theta(static_cast<const double2 *>(w[i].phi), s.trial, s.M, s.Na, s.Nb, s.W, s.theta,
                                s.logo_new, s.stat_new, nullptr, st, s.opart, s.ospart),
              "overlap kernel");
    AFQMC_HIP(launch_force_bias_gemm(s, s.theta, s.W, st), "force-bias kernel");
    s.fb_slices = s.fb_ksplit;
    AFQMC_HIP(launch_fb_energy_epilogue(s, s.W, static_cast<double2 *>(vbias_out[i]), s.fb_slices, st),
              "force-bias epilogue");
  }
  return AFQMC_OK;
}

afqmc_status afqmc_cv_collect(afqmc_ctx *ctx, const afqmc_walkers *w, double *const *feat_out, void *const *ek_out,
                              void *hip_stream) {
  if (!ctx || !w || !feat_out || !ek_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers or outputs");
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    if (!w[i].phi || !feat_out[i] || !ek_out[i]) return fail(AFQMC_ERR_ARG, "NULL phi or output");
  }
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    {
      Phase ph(ctx, AFQMC_PH_OVERLAP, ls);
      AFQMC_HIP(launch_ovlp_theta(static_cast<const double2 *>(w[i].phi), s.trial, s.M, s.Na, s.Nb, s.W, s.theta,
                                  s.logo_new, s.stat_new, nullptr, ls, s.opart, s.ospart),
                "overlap kernel");
    }
    {
      Phase ph(ctx, AFQMC_PH_FORCE_BIAS, ls);
      AFQMC_HIP(launch_force_bias_gemm(s, s.theta, s.W, ls), "force-bias kernel");
    }
    s.fb_slices = s.fb_ksplit;
    {
      Phase ph(ctx, AFQMC_PH_ENERGY_1B, ls);
      AFQMC_HIP(launch_energy_e1(s, s.theta, s.W, ls), "one-body energy kernel");
    }
    {
      Phase ph(ctx, AFQMC_PH_FB_EPILOGUE, ls);
      AFQMC_HIP(launch_fb_energy_epilogue(s, s.W, nullptr, s.fb_slices, ls), "Coulomb epilogue");
    }
    {
      Phase ph(ctx, AFQMC_PH_CV, ls);
      AFQMC_HIP(launch_cv_features(s, s.W, feat_out[i], ls), "feature kernel");
    }
    afqmc_status r = exchange_sys(ctx, s, s.theta, s.W, nullptr, ls);
    if (r != AFQMC_OK) return r;
    AFQMC_HIP(launch_cv_ek(s, s.W, static_cast<double2 *>(ek_out[i]), ls), "exchange sum kernel");
    return AFQMC_OK;
  });
}

}  // extern "C"

namespace {

System *cv_system(afqmc_ctx *ctx, int32_t isys) {
  if (!ctx || isys < 0 || isys >= (int)ctx->sys.size()) return nullptr;
  return &ctx->sys[isys];
}

// Device workspace of a synchronous call: freed after the stream has finished.
struct Workspace {
  std::vector<void *> ptrs;
  hipStream_t st = nullptr;
  ~Workspace() {
    if (!ptrs.empty()) (void)hipStreamSynchronize(st);
    for (void *p : ptrs) (void)hipFree(p);
  }
  template <class T>
  bool get(T **p, size_t count) {
    void *q = nullptr;
    if (hipMalloc(&q, (count ? count : 1) * sizeof(T)) != hipSuccess) {
      (void)hipGetLastError();
      return false;
    }
    ptrs.push_back(q);
    *p = static_cast<T *>(q);
    return true;
  }
};

}  // namespace

extern "C" {

afqmc_status afqmc_cv_train(afqmc_ctx *ctx, int32_t isys, const double *feat, const void *ek, int64_t n,
                            int32_t epochs, int32_t batch, double lr, double *loss_out, void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp || !feat || !ek) return fail(AFQMC_ERR_ARG, "NULL context, inputs or bad system index");
  if (n < 2 || epochs < 0 || batch < 1 || !(lr > 0.0) || n > (int64_t)1 << 30)
    return fail(AFQMC_ERR_ARG, "need n >= 2, epochs >= 0, batch >= 1 and lr > 0");
  System &s = *sp;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  const long nb_max = std::min<long>(batch, n);
  Workspace ws;
  ws.st = st;
  float *X = nullptr, *T = nullptr, *part = nullptr, *grad = nullptr;
  double *lpart = nullptr, *loss = nullptr;
  if (!ws.get(&X, (size_t)n * kCvFeatures) || !ws.get(&T, (size_t)n * 2) ||
      !ws.get(&part, (size_t)cv_grad_workgroups(nb_max) * kCvParams) || !ws.get(&grad, kCvParams) ||
      !ws.get(&lpart, (size_t)cv_grad_workgroups(nb_max)) || !ws.get(&loss, (size_t)std::max(1, epochs)))
    return fail(AFQMC_ERR_OOM, "device allocation failed (training workspace)");
  AFQMC_HIP(launch_cv_stats(feat, static_cast<const double2 *>(ek), n, s.cv_norm, st), "statistics kernel");
  AFQMC_HIP(launch_cv_standardise(feat, static_cast<const double2 *>(ek), n, s.cv_norm, X, T, st),
            "standardise kernel");
  AFQMC_HIP(launch_cv_zero(s.cv_m, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(s.cv_v, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(loss, (size_t)std::max(1, epochs) * sizeof(double), st), "zero fill");
  long t = 0;
  for (int e = 0; e < epochs; ++e)
    for (long b0 = 0; b0 < n; b0 += batch) {
      const long nb = std::min<long>(batch, n - b0);
      AFQMC_HIP(launch_cv_grad(s.cv_params, X, T, b0, nb, part, lpart, grad, (double)nb / (double)n, loss + e, st),
                "network gradient kernel");
      AFQMC_HIP(launch_cv_adam(s.cv_params, grad, s.cv_m, s.cv_v, lr, ++t, st), "Adam kernel");
    }
  if (loss_out && epochs > 0)
    AFQMC_HIP(hipMemcpyAsync(loss_out, loss, (size_t)epochs * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  AFQMC_HIP(hipStreamSynchronize(st), "training");
  return AFQMC_OK;
}

afqmc_status afqmc_cv_train_noalloc(afqmc_ctx *ctx, int32_t isys, const double *feat, const void *ek, int64_t n,
                                    int32_t epochs, int32_t batch, double lr, double *loss_out, void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp || !feat || !ek) return fail(AFQMC_ERR_ARG, "NULL context, inputs or bad system index");
  if (n < 2 || epochs < 0 || batch < 1 || !(lr > 0.0))
    return fail(AFQMC_ERR_ARG, "need n >= 2, epochs >= 0, batch >= 1 and lr > 0");
  if (n > kNoAllocMaxSamples || std::min<int64_t>(batch, n) > kNoAllocMaxBatch)
    return fail(AFQMC_ERR_UNSUPPORTED, "afqmc_cv_train_noalloc takes at most " + std::to_string(kNoAllocMaxSamples) +
                                           " samples and minibatches of at most " +
                                           std::to_string(kNoAllocMaxBatch) + " (got n = " + std::to_string(n) +
                                           ", batch = " + std::to_string(batch) + ")");
  unsigned char *base = scratch_address(ctx->device);
  if (!base) return fail(AFQMC_ERR_HIP, "the no-allocation workspace has no address on this device");
  System &s = *sp;
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  float *X = reinterpret_cast<float *>(base + kNaX), *T = reinterpret_cast<float *>(base + kNaT);
  float *part = reinterpret_cast<float *>(base + kNaPart), *grad = reinterpret_cast<float *>(base + kNaGrad);
  double *lpart = reinterpret_cast<double *>(base + kNaLpart);
  // nothing in the workspace accumulates: every kernel below writes what it
  // reads later in this call; the loss accumulates in the caller's buffer
  AFQMC_HIP(launch_cv_stats(feat, static_cast<const double2 *>(ek), n, s.cv_norm, st), "statistics kernel");
  AFQMC_HIP(launch_cv_standardise(feat, static_cast<const double2 *>(ek), n, s.cv_norm, X, T, st),
            "standardise kernel");
  AFQMC_HIP(launch_cv_zero(s.cv_m, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(s.cv_v, kCvParams * sizeof(float), st), "zero fill");
  if (loss_out && epochs > 0) AFQMC_HIP(launch_cv_zero(loss_out, (size_t)epochs * sizeof(double), st), "zero fill");
  long t = 0;
  for (int e = 0; e < epochs; ++e)
    for (long b0 = 0; b0 < n; b0 += batch) {
      const long nb = std::min<long>(batch, n - b0);
      AFQMC_HIP(launch_cv_grad(s.cv_params, X, T, b0, nb, part, lpart, grad, (double)nb / (double)n,
                               loss_out ? loss_out + e : nullptr, st),
                "network gradient kernel");
      AFQMC_HIP(launch_cv_adam(s.cv_params, grad, s.cv_m, s.cv_v, lr, ++t, st), "Adam kernel");
    }
  return AFQMC_OK;
}

afqmc_status afqmc_cv_set_params(afqmc_ctx *ctx, int32_t isys, const float *params, const double *norm,
                                 void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp) return fail(AFQMC_ERR_ARG, "NULL context or bad system index");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (params)
    AFQMC_HIP(hipMemcpyAsync(sp->cv_params, params, kCvParams * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
  if (norm) AFQMC_HIP(hipMemcpyAsync(sp->cv_norm, norm, kCvNorm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  AFQMC_HIP(launch_cv_zero(sp->cv_m, kCvParams * sizeof(float), st), "zero fill");
  AFQMC_HIP(launch_cv_zero(sp->cv_v, kCvParams * sizeof(float), st), "zero fill");
  return AFQMC_OK;
}

afqmc_status afqmc_cv_get_params(afqmc_ctx *ctx, int32_t isys, float *params, double *norm, void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp) return fail(AFQMC_ERR_ARG, "NULL context or bad system index");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (params)
    AFQMC_HIP(hipMemcpyAsync(params, sp->cv_params, kCvParams * sizeof(float), hipMemcpyDeviceToDevice, st), "copy");
  if (norm) AFQMC_HIP(hipMemcpyAsync(norm, sp->cv_norm, kCvNorm * sizeof(double), hipMemcpyDeviceToDevice, st), "copy");
  return AFQMC_OK;
}

afqmc_status afqmc_cv_predict(afqmc_ctx *ctx, int32_t isys, const double *feat, int64_t n, void *f_out,
                              void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp || !feat || !f_out) return fail(AFQMC_ERR_ARG, "NULL context, inputs or bad system index");
  if (n < 0 || n > (int64_t)1 << 30) return fail(AFQMC_ERR_ARG, "bad sample count");
  AFQMC_HIP(launch_cv_predict(*sp, feat, n, static_cast<double2 *>(f_out), static_cast<hipStream_t>(hip_stream)),
            "network kernel");
  return AFQMC_OK;
}

afqmc_status afqmc_cv_loss_grad(afqmc_ctx *ctx, int32_t isys, const float *x, const float *t, int64_t n,
                                float *grad_out, double *loss_out, void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp || !x || !t || !grad_out || !loss_out) return fail(AFQMC_ERR_ARG, "NULL argument or bad system index");
  if (n < 1 || n > (int64_t)1 << 30) return fail(AFQMC_ERR_ARG, "bad sample count");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  Workspace ws;
  ws.st = st;
  float *part = nullptr;
  double *lpart = nullptr;
  if (!ws.get(&part, (size_t)cv_grad_workgroups(n) * kCvParams) || !ws.get(&lpart, (size_t)cv_grad_workgroups(n)))
    return fail(AFQMC_ERR_OOM, "device allocation failed (gradient workspace)");
  AFQMC_HIP(launch_cv_zero(loss_out, sizeof(double), st), "zero fill");
  AFQMC_HIP(launch_cv_grad(sp->cv_params, x, t, 0, n, part, lpart, grad_out, 1.0, loss_out, st),
            "network gradient kernel");
  AFQMC_HIP(hipStreamSynchronize(st), "gradient");
  return AFQMC_OK;
}

afqmc_status afqmc_cv_state(afqmc_ctx *ctx, int32_t isys, void *f_out, int32_t *subset_out, uint64_t *call_out,
                            void *hip_stream) {
  System *sp = cv_system(ctx, isys);
  if (!sp) return fail(AFQMC_ERR_ARG, "NULL context or bad system index");
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  if (f_out)
    AFQMC_HIP(hipMemcpyAsync(f_out, sp->cv_f, (size_t)sp->W * sizeof(double2), hipMemcpyDeviceToDevice, st), "copy");
  if (subset_out)
    AFQMC_HIP(hipMemcpyAsync(subset_out, sp->cv_sel, (size_t)sp->cv_k * sizeof(int32_t), hipMemcpyDeviceToDevice, st),
              "copy");
  if (call_out)
    AFQMC_HIP(hipMemcpyAsync(call_out, sp->cv_counter + 1, sizeof(uint64_t), hipMemcpyDeviceToDevice, st), "copy");
  return AFQMC_OK;
}

afqmc_status afqmc_population_control(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *u,
                                      int32_t *const *parents_out, void *hip_stream) {
  if (!ctx || !w || !u) return fail(AFQMC_ERR_ARG, "NULL context, walkers or offsets");
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!u[i]) return fail(AFQMC_ERR_ARG, "offset of system " + std::to_string(i) + " is NULL");
  }
  invalidate_caches(ctx);
  hipStream_t st = static_cast<hipStream_t>(hip_stream);
  return for_each_system(ctx, st, [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    AFQMC_HIP(launch_comb(s, w[i].weight, static_cast<double2 *>(w[i].phi), static_cast<double2 *>(w[i].log_ovlp),
                          w[i].flags, u[i], parents_out ? parents_out[i] : nullptr, ls),
              "population control kernels");
    return AFQMC_OK;
  });
}

afqmc_status afqmc_set_e_shift(afqmc_ctx *ctx, int32_t isys, double e_shift, void *hip_stream) {
  if (!ctx || isys < 0 || isys >= (int)ctx->sys.size()) return fail(AFQMC_ERR_ARG, "NULL context or bad index");
  if (!std::isfinite(e_shift)) return fail(AFQMC_ERR_ARG, "e_shift must be finite");
  // the weight kernels read E_T from device memory: recorded steps stay valid
  AFQMC_HIP(launch_set_e_shift(ctx->sys[isys], e_shift, static_cast<hipStream_t>(hip_stream)), "energy-shift kernel");
  return AFQMC_OK;
}

static afqmc_status check_amplitudes(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *log_amp) {
  if (!log_amp) return fail(AFQMC_ERR_ARG, "NULL log-amplitudes");
  for (size_t i = 0; i < ctx->sys.size(); ++i) {
    afqmc_status r = check_walkers(w[i], (int)i);
    if (r != AFQMC_OK) return r;
    if (!log_amp[i]) return fail(AFQMC_ERR_ARG, "log-amplitudes of system " + std::to_string(i) + " are NULL");
  }
  return AFQMC_OK;
}

afqmc_status afqmc_free_propagate(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x,
                                  void *const *log_amp, void *hip_stream) {
  if (!ctx || !w || !x) return fail(AFQMC_ERR_ARG, "NULL context, walkers or fields");
  afqmc_status r = check_amplitudes(ctx, w, log_amp);
  if (r != AFQMC_OK) return r;
  for (size_t i = 0; i < ctx->sys.size(); ++i)
    if (!x[i]) return fail(AFQMC_ERR_ARG, "fields of system " + std::to_string(i) + " are NULL");
  invalidate_caches(ctx);
  return for_each_system(ctx, static_cast<hipStream_t>(hip_stream), [&](int i, hipStream_t ls) {
    return free_propagate_sys(ctx, ctx->sys[i], w[i], x[i], static_cast<double2 *>(log_amp[i]), false, ls);
  });
}

afqmc_status afqmc_free_estimator(afqmc_ctx *ctx, const afqmc_walkers *w, void *const *log_amp, void *const *e_in,
                                  double *est_out, void *hip_stream) {
  if (!ctx || !w || !e_in || !est_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers, energies or est_out");
  afqmc_status r = check_amplitudes(ctx, w, log_amp);
  if (r != AFQMC_OK) return r;
  for (size_t i = 0; i < ctx->sys.size(); ++i)
    if (!e_in[i]) return fail(AFQMC_ERR_ARG, "energies of system " + std::to_string(i) + " are NULL");
  return for_each_system(ctx, static_cast<hipStream_t>(hip_stream), [&](int i, hipStream_t ls) {
    Phase ph(ctx, AFQMC_PH_COMBINE, ls);
    AFQMC_HIP(launch_free_estimator(w[i].weight, w[i].flags, static_cast<const double2 *>(log_amp[i]),
                                    static_cast<const double2 *>(e_in[i]), ctx->sys[i].W,
                                    est_out + (size_t)AFQMC_FREE_EST * i, ls),
              "estimator kernel");
    return AFQMC_OK;
  });
}

afqmc_status afqmc_free_step(afqmc_ctx *ctx, const afqmc_walkers *w, const double *const *x, void *const *log_amp,
                             void *const *e_out, double *est_out, uint32_t flags, void *hip_stream) {
  if (!ctx || !w || !x || !e_out) return fail(AFQMC_ERR_ARG, "NULL context, walkers, fields or e_out");
  if (flags & ~(uint32_t)AFQMC_STEP_REORTHO) return fail(AFQMC_ERR_ARG, "unknown free-step flags");
  afqmc_status r = check_amplitudes(ctx, w, log_amp);
  if (r != AFQMC_OK) return r;
  for (size_t i = 0; i < ctx->sys.size(); ++i)
    if (!x[i] || !e_out[i]) return fail(AFQMC_ERR_ARG, "NULL fields or e_out of system " + std::to_string(i));
  invalidate_caches(ctx);
  return for_each_system(ctx, static_cast<hipStream_t>(hip_stream), [&](int i, hipStream_t ls) {
    System &s = ctx->sys[i];
    double2 *amp = static_cast<double2 *>(log_amp[i]);
    double2 *e = static_cast<double2 *>(e_out[i]);
    afqmc_status rr = free_propagate_sys(ctx, s, w[i], x[i], amp, true, ls);
    if (rr != AFQMC_OK) return rr;
    if (flags & AFQMC_STEP_REORTHO) {
      Phase ph(ctx, AFQMC_PH_REORTHO, ls);
      AFQMC_HIP(launch_mgs(static_cast<double2 *>(w[i].phi), s.M, s.Na, s.Nb, s.W,
                           static_cast<double2 *>(w[i].log_ovlp), ls, reinterpret_cast<double *>(s.opart)),
                "Gram-Schmidt kernel");
    }
    rr = local_energy_sys(ctx, s, static_cast<const double2 *>(w[i].phi), s.W, e, nullptr, w[i].weight, ls, true);
    if (rr != AFQMC_OK) return rr;
    if (est_out) {
      Phase ph(ctx, AFQMC_PH_COMBINE, ls);
      AFQMC_HIP(launch_free_estimator(w[i].weight, w[i].flags, amp, e, s.W, est_out + (size_t)AFQMC_FREE_EST * i, ls),
                "estimator kernel");
    }
    return AFQMC_OK;
  });
}

afqmc_status afqmc_set_timing(afqmc_ctx *ctx, int32_t enable) {
  if (!ctx) return fail(AFQMC_ERR_ARG, "NULL context");
  fold_timings(ctx);
  ctx->timing = enable != 0;
  if (ctx->timing)
    for (int i = 0; i < AFQMC_NPHASES; ++i) {
      ctx->ph_ms[i] = 0.0;
      ctx->ph_count[i] = 0;
    }
  return AFQMC_OK;
}

afqmc_status afqmc_get_timings(afqmc_ctx *ctx, afqmc_timings *out) {
  if (!ctx || !out) return fail(AFQMC_ERR_ARG, "NULL context or out");
  fold_timings(ctx);
  for (int i = 0; i < AFQMC_NPHASES; ++i) {
    out->ms[i] = ctx->ph_ms[i];
    out->count[i] = ctx->ph_count[i];
  }
  return AFQMC_OK;
}

afqmc_status afqmc_get_info(const afqmc_ctx *ctx, int32_t isys, afqmc_info *out) {
  if (!ctx || !out) return fail(AFQMC_ERR_ARG, "NULL context or out");
  if (isys < 0 || isys >= (int)ctx->sys.size()) return fail(AFQMC_ERR_ARG, "system index out of range");
  const System &s = ctx->sys[isys];
  out->e_hf = s.e_hf;
  double et = s.e_shift;
  if (hipDeviceSynchronize() != hipSuccess || hipMemcpy(&et, s.eshift, sizeof(double), hipMemcpyDeviceToHost) != hipSuccess)
    return fail(AFQMC_ERR_HIP, "reading the energy shift");
  out->e_shift = et;
  out->const_c = s.const_c;
  out->device_bytes = s.bytes;
  out->exchange_tile = s.ex_mfma ? s.ex_plan[s.Na > 0 ? 0 : 1].WX : 0;
  out->exchange_order = s.ex_mfma ? s.ex_group : -1;
  out->lane = ctx->lanes.empty() ? -1 : ctx->lane_of[isys];
  out->graph_captures = ctx->graph_captures;
  out->graph_replays = ctx->graph_replays;
  out->cv_subset = s.ex_mode == AFQMC_EX_CV ? s.cv_k : 0;
  out->vhs_tile = s.use_mfma_gemm && !s.prop32 ? s.vhs_shape : -1;
  out->taylor_tile = s.prop32 || taylor_walker_split(s) ? s.taylor_shape : -1;
  out->reserved_info = 0;
  return AFQMC_OK;
}

void afqmc_destroy(afqmc_ctx *ctx) {
  if (!ctx) return;
  release(ctx);
  delete ctx;
}

}  // extern "C"
