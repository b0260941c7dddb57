"""Python binding of libafqmc (the C ABI declared in include/afqmc.h).

Argument marshalling only: every step of the walker update runs in the
library's HIP kernels.  torch supplies device memory and the stream; numpy
arrays supply the host-side Hamiltonian at set-up.  If the library is not
built, every entry point raises: there is no CPU fallback.

Entry points carry the C names without the ``afqmc_`` prefix:
setup_hamiltonian, propagate, local_energy, reorthogonalize, overlap,
greens_function, force_bias, get_info, destroy, last_error.
"""
from __future__ import annotations

import ctypes
import dataclasses
import itertools
import os
from typing import Sequence

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libafqmc.so")

OK, ERR_ARG, ERR_OOM, ERR_HIP, ERR_UNSUPPORTED = 0, 1, 2, 3, 4
FP64, FP32_CONTRACT, BF16X3_CONTRACT, BF16X2_CONTRACT, FP16_TSPLIT_CONTRACT, BF16_TSPLIT_CONTRACT = 0, 1, 2, 3, 4, 5
W_SINGULAR, W_NONFINITE, W_DEAD = 1, 2, 4
EX_FULL, EX_CV = 0, 1
_STATUS = {0: "OK", 1: "ERR_ARG", 2: "ERR_OOM", 3: "ERR_HIP", 4: "ERR_UNSUPPORTED"}


class AfqmcError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS.get(status, status)}: {message}")
        self.status = status


class SystemDesc(ctypes.Structure):
    _fields_ = [("nbasis", ctypes.c_int32), ("nalpha", ctypes.c_int32), ("nbeta", ctypes.c_int32),
                ("nchol", ctypes.c_int32), ("nwalkers", ctypes.c_int32),
                ("h1", ctypes.c_void_p), ("chol", ctypes.c_void_p), ("ecore", ctypes.c_double),
                ("trial", ctypes.c_void_p), ("dt", ctypes.c_double), ("chol_gen", ctypes.c_int32),
                ("reserved_desc", ctypes.c_int32), ("gen_seed", ctypes.c_uint64), ("gen_tau", ctypes.c_double),
                ("gen_scale", ctypes.c_double)]


class Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("taylor_order", ctypes.c_int32),
                ("fb_cap", ctypes.c_double), ("e_shift", ctypes.c_double),
                ("mem_limit_bytes", ctypes.c_uint64), ("streams", ctypes.c_int32), ("use_graph", ctypes.c_int32),
                ("tune", ctypes.c_int32), ("ex_mode", ctypes.c_int32), ("cv_fraction", ctypes.c_double),
                ("cv_seed", ctypes.c_uint64), ("prop_precision", ctypes.c_int32), ("deterministic", ctypes.c_int32),
                ("tune_cache", ctypes.c_char_p), ("reserved", ctypes.c_int32 * 8)]


class CWalkers(ctypes.Structure):
    _fields_ = [("phi", ctypes.c_void_p), ("weight", ctypes.c_void_p),
                ("log_ovlp", ctypes.c_void_p), ("flags", ctypes.c_void_p)]


class Info(ctypes.Structure):
    _fields_ = [("e_hf", ctypes.c_double), ("e_shift", ctypes.c_double),
                ("const_c", ctypes.c_double), ("device_bytes", ctypes.c_uint64),
                ("exchange_tile", ctypes.c_int32), ("exchange_order", ctypes.c_int32), ("lane", ctypes.c_int32),
                ("graph_captures", ctypes.c_int64), ("graph_replays", ctypes.c_int64),
                ("cv_subset", ctypes.c_int32), ("vhs_tile", ctypes.c_int32), ("taylor_tile", ctypes.c_int32),
                ("reserved_info", ctypes.c_int32)]


PHASES = ("overlap", "force_bias", "fb_epilogue", "vhs", "one_body", "taylor", "weight",
          "energy_1b", "exchange", "combine", "reortho", "operands", "cv")


class Timings(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * len(PHASES)), ("count", ctypes.c_int64 * len(PHASES))]


STEP_REORTHO, STEP_FRESH = 1, 2
BLOCK_FEEDBACK = 4
REBLOCK_LEVELS = 64


class ReblockResult(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("mean", ctypes.c_double), ("nlevels", ctypes.c_int32),
                ("optimal", ctypes.c_int32), ("count", ctypes.c_int64 * REBLOCK_LEVELS),
                ("level_mean", ctypes.c_double * REBLOCK_LEVELS), ("std_err", ctypes.c_double * REBLOCK_LEVELS),
                ("std_err_err", ctypes.c_double * REBLOCK_LEVELS)]

EXPORTS = ("afqmc_default_options", "afqmc_setup_hamiltonian", "afqmc_propagate",
           "afqmc_local_energy", "afqmc_reorthogonalize", "afqmc_step", "afqmc_overlap",
           "afqmc_greens_function", "afqmc_force_bias", "afqmc_get_info",
           "afqmc_set_timing", "afqmc_get_timings", "afqmc_destroy", "afqmc_last_error",
           "afqmc_cv_collect", "afqmc_cv_train", "afqmc_cv_set_params", "afqmc_cv_get_params",
           "afqmc_cv_predict", "afqmc_cv_loss_grad", "afqmc_cv_state", "afqmc_population_control",
           "afqmc_set_e_shift", "afqmc_free_propagate", "afqmc_free_estimator", "afqmc_free_step",
           "afqmc_run_block", "afqmc_reblock", "afqmc_cv_train_noalloc")
CV_NFEAT, CV_NPARAMS, CV_NNORM = 10, 18178, 24
CV_NOALLOC_MAX_SAMPLES, CV_NOALLOC_MAX_BATCH = 65536, 512
FREE_EST = 10

_lib = None


def load_library() -> ctypes.CDLL:
    """Load libafqmc.so from the package directory (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise AfqmcError(ERR_UNSUPPORTED, f"{LIB_PATH} is not built; run "
                         "`python -m paper_2406_16238_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    pp = ctypes.POINTER(ctypes.c_void_p)
    sigs = {
        "afqmc_default_options": ([ctypes.POINTER(Options)], ctypes.c_int),
        "afqmc_setup_hamiltonian": ([ctypes.POINTER(SystemDesc), ctypes.c_int32, ctypes.POINTER(Options), P,
                                     ctypes.POINTER(P)], ctypes.c_int),
        "afqmc_propagate": ([P, ctypes.POINTER(CWalkers), pp, P], ctypes.c_int),
        "afqmc_local_energy": ([P, ctypes.POINTER(CWalkers), pp, P, P], ctypes.c_int),
        "afqmc_reorthogonalize": ([P, ctypes.POINTER(CWalkers), P], ctypes.c_int),
        "afqmc_step": ([P, ctypes.POINTER(CWalkers), pp, pp, P, ctypes.c_uint32, P], ctypes.c_int),
        "afqmc_overlap": ([P, ctypes.POINTER(CWalkers), P], ctypes.c_int),
        "afqmc_greens_function": ([P, ctypes.POINTER(CWalkers), pp, P], ctypes.c_int),
        "afqmc_force_bias": ([P, ctypes.POINTER(CWalkers), pp, P], ctypes.c_int),
        "afqmc_get_info": ([P, ctypes.c_int32, ctypes.POINTER(Info)], ctypes.c_int),
        "afqmc_set_timing": ([P, ctypes.c_int32], ctypes.c_int),
        "afqmc_get_timings": ([P, ctypes.POINTER(Timings)], ctypes.c_int),
        "afqmc_destroy": ([P], None),
        "afqmc_last_error": ([], ctypes.c_char_p),
        "afqmc_cv_collect": ([P, ctypes.POINTER(CWalkers), pp, pp, P], ctypes.c_int),
        "afqmc_cv_train": ([P, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                            ctypes.c_double, P, P], ctypes.c_int),
        "afqmc_cv_train_noalloc": ([P, ctypes.c_int32, P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.c_double, P, P], ctypes.c_int),
        "afqmc_cv_set_params": ([P, ctypes.c_int32, P, P, P], ctypes.c_int),
        "afqmc_cv_get_params": ([P, ctypes.c_int32, P, P, P], ctypes.c_int),
        "afqmc_cv_predict": ([P, ctypes.c_int32, P, ctypes.c_int64, P, P], ctypes.c_int),
        "afqmc_cv_loss_grad": ([P, ctypes.c_int32, P, P, ctypes.c_int64, P, P, P], ctypes.c_int),
        "afqmc_cv_state": ([P, ctypes.c_int32, P, P, P, P], ctypes.c_int),
        "afqmc_population_control": ([P, ctypes.POINTER(CWalkers), pp, pp, P], ctypes.c_int),
        "afqmc_set_e_shift": ([P, ctypes.c_int32, ctypes.c_double, P], ctypes.c_int),
        "afqmc_run_block": ([P, ctypes.POINTER(CWalkers), pp, ctypes.c_int32, ctypes.c_int64, ctypes.c_int32, pp,
                             pp, pp, ctypes.c_uint32, P], ctypes.c_int),
        "afqmc_reblock": ([P, ctypes.c_int64, ctypes.POINTER(ReblockResult)], ctypes.c_int),
        "afqmc_free_propagate": ([P, ctypes.POINTER(CWalkers), pp, pp, P], ctypes.c_int),
        "afqmc_free_estimator": ([P, ctypes.POINTER(CWalkers), pp, pp, P, P], ctypes.c_int),
        "afqmc_free_step": ([P, ctypes.POINTER(CWalkers), pp, pp, pp, P, ctypes.c_uint32, P], ctypes.c_int),
    }
    for name, (args, res) in sigs.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    _lib = lib
    return lib


def last_error() -> str:
    return load_library().afqmc_last_error().decode()


def _check(status: int):
    if status != OK:
        raise AfqmcError(status, last_error())


def default_options(**overrides) -> Options:
    o = Options()
    _check(load_library().afqmc_default_options(ctypes.byref(o)))
    for k, v in overrides.items():
        setattr(o, k, v)
    return o


def _stream_handle(stream) -> int:
    import torch
    if stream is None:
        stream = torch.cuda.current_stream()
    return int(stream.cuda_stream)


@dataclasses.dataclass
class CholGen:
    """The device-side synthetic Cholesky recipe (chol_gen = 1): seed, decay
    length and scale, for G vectors."""

    nchol: int
    seed: int
    tau: float
    scale: float


@dataclasses.dataclass
class SystemInput:
    """Host-side description of one system (float64 numpy arrays).  `chol` is
    either the [G, M, M] array or a CholGen (the library draws L on the device)."""

    h1: np.ndarray
    chol: "np.ndarray | CholGen"
    ecore: float
    trial: np.ndarray
    nalpha: int
    nbeta: int
    nwalkers: int
    dt: float

    @property
    def nbasis(self):
        return self.h1.shape[0]

    @property
    def nchol(self):
        return self.chol.nchol if isinstance(self.chol, CholGen) else self.chol.shape[0]


_walker_ids = itertools.count(1)


@dataclasses.dataclass
class Walkers:
    """Caller-owned walker state of one system (torch tensors on the GPU).

    `ident` tells walker sets apart: step() and run_block() ask the library to
    recompute its cached Green's function (AFQMC_STEP_FRESH) whenever the sets
    differ from those of the context's previous step, even when new tensors
    happen to reuse the old ones' device addresses."""

    phi: "object"        # complex128 [W, M, Na+Nb]
    weight: "object"     # float64 [W]
    log_ovlp: "object"   # complex128 [W]
    flags: "object"      # int32 [W] (bit pattern of the library's uint32 flags)
    ident: int = dataclasses.field(default_factory=lambda: next(_walker_ids), compare=False)

    def c_struct(self) -> CWalkers:
        import torch
        for name, t, dt in (("phi", self.phi, torch.complex128), ("weight", self.weight, torch.float64),
                            ("log_ovlp", self.log_ovlp, torch.complex128), ("flags", self.flags, torch.int32)):
            if t.dtype != dt or not t.is_cuda or not t.is_contiguous():
                raise ValueError(f"walker field {name} must be a contiguous {dt} CUDA tensor")
        return CWalkers(self.phi.data_ptr(), self.weight.data_ptr(), self.log_ovlp.data_ptr(),
                        self.flags.data_ptr())

    @staticmethod
    def from_numpy(phi: np.ndarray, device="cuda"):
        import torch
        w = phi.shape[0]
        return Walkers(torch.as_tensor(np.ascontiguousarray(phi, np.complex128), device=device),
                       torch.ones(w, dtype=torch.float64, device=device),
                       torch.zeros(w, dtype=torch.complex128, device=device),
                       torch.zeros(w, dtype=torch.int32, device=device))


class Context:
    """Owns an afqmc_ctx; destroyed by close() or garbage collection."""

    def __init__(self, handle: int, systems: Sequence[SystemInput], options: Options):
        self.handle = ctypes.c_void_p(handle)
        self.systems = list(systems)
        self.options = options
        self.last_stepped = None   # idents of the walker sets of the previous step or block

    def stepping(self, walkers) -> bool:
        """Records the walker sets about to be stepped; True when they are the
        previous step's (the library's cache may apply)."""
        ids = tuple(w.ident for w in (walkers if isinstance(walkers, (list, tuple)) else [walkers]))
        same = ids == self.last_stepped
        self.last_stepped = ids
        return same

    @property
    def nsys(self):
        return len(self.systems)

    def close(self):
        if self.handle is not None and self.handle.value:
            load_library().afqmc_destroy(self.handle)
        self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def setup_hamiltonian(systems: Sequence[SystemInput] | SystemInput, options: Options | None = None,
                      stream=None) -> Context:
    """afqmc_setup_hamiltonian: copy and derive the Hamiltonian on the device."""
    lib = load_library()
    if isinstance(systems, SystemInput):
        systems = [systems]
    keep = []
    descs = (SystemDesc * len(systems))()
    for i, s in enumerate(systems):
        h1 = np.ascontiguousarray(s.h1, np.float64)
        trial = np.ascontiguousarray(s.trial, np.float64)
        m = h1.shape[0]
        gen = s.chol if isinstance(s.chol, CholGen) else None
        if gen is None:
            chol = np.ascontiguousarray(s.chol, np.float64)
            if chol.ndim != 3 or chol.shape[1:] != (m, m):
                raise ValueError(f"system {i}: inconsistent array shapes")
            keep.append(chol)
        if h1.shape != (m, m) or trial.shape != (m, s.nalpha + s.nbeta):
            raise ValueError(f"system {i}: inconsistent array shapes")
        keep += [h1, trial]
        descs[i] = SystemDesc(m, s.nalpha, s.nbeta, s.nchol, s.nwalkers, h1.ctypes.data,
                              None if gen else chol.ctypes.data, float(s.ecore), trial.ctypes.data, float(s.dt),
                              1 if gen else 0, 0, gen.seed if gen else 0, gen.tau if gen else 0.0,
                              gen.scale if gen else 0.0)
    opt = options if options is not None else default_options()
    handle = ctypes.c_void_p()
    st = _stream_handle(stream) if stream is not False else 0
    _check(lib.afqmc_setup_hamiltonian(descs, len(systems), ctypes.byref(opt), st, ctypes.byref(handle)))
    return Context(handle.value, systems, opt)


def _walker_array(ctx: Context, walkers):
    if isinstance(walkers, Walkers):
        walkers = [walkers]
    if len(walkers) != ctx.nsys:
        raise ValueError(f"expected {ctx.nsys} walker sets, got {len(walkers)}")
    arr = (CWalkers * ctx.nsys)()
    for i, (w, s) in enumerate(zip(walkers, ctx.systems)):
        shape = (s.nwalkers, s.nbasis, s.nalpha + s.nbeta)
        if tuple(w.phi.shape) != shape or tuple(w.weight.shape) != (s.nwalkers,) \
                or tuple(w.log_ovlp.shape) != (s.nwalkers,) or tuple(w.flags.shape) != (s.nwalkers,):
            raise ValueError(f"system {i}: walker tensors must have shape {shape} / ({s.nwalkers},)")
        arr[i] = w.c_struct()
    return arr


def _ptr_array(ctx: Context, tensors, shapes, dtype):
    if not isinstance(tensors, (list, tuple)):
        tensors = [tensors]
    if len(tensors) != ctx.nsys:
        raise ValueError(f"expected {ctx.nsys} buffers, got {len(tensors)}")
    arr = (ctypes.c_void_p * ctx.nsys)()
    for i, (t, shp) in enumerate(zip(tensors, shapes)):
        if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shp):
            raise ValueError(f"buffer {i} must be a contiguous {dtype} CUDA tensor of shape {shp}")
        arr[i] = t.data_ptr()
    return arr


def propagate(ctx: Context, walkers, x, stream=None):
    """afqmc_propagate: one phaseless time step; x is [W, G] float64 per system."""
    import torch
    w = _walker_array(ctx, walkers)
    xs = _ptr_array(ctx, x, [(s.nwalkers, s.nchol) for s in ctx.systems], torch.float64)
    _check(load_library().afqmc_propagate(ctx.handle, w, xs, _stream_handle(stream)))


def local_energy(ctx: Context, walkers, e_out, est_out=None, stream=None):
    """afqmc_local_energy: e_out complex128 [W, 3] per system; est_out float64 [nsys, 4] or None."""
    import torch
    w = _walker_array(ctx, walkers)
    es = _ptr_array(ctx, e_out, [(s.nwalkers, 3) for s in ctx.systems], torch.complex128)
    est = None
    if est_out is not None:
        if est_out.dtype != torch.float64 or not est_out.is_cuda or tuple(est_out.shape) != (ctx.nsys, 4):
            raise ValueError("est_out must be a float64 CUDA tensor of shape (nsys, 4)")
        est = est_out.data_ptr()
    _check(load_library().afqmc_local_energy(ctx.handle, w, es, est, _stream_handle(stream)))


def step(ctx: Context, walkers, x, e_out, est_out=None, reortho=False, fresh=False, stream=None):
    """afqmc_step: propagate, optionally re-orthogonalise, then local energy, with
    one overlap/LU and one force-bias contraction per step."""
    import torch
    w = _walker_array(ctx, walkers)
    xs = _ptr_array(ctx, x, [(s.nwalkers, s.nchol) for s in ctx.systems], torch.float64)
    es = _ptr_array(ctx, e_out, [(s.nwalkers, 3) for s in ctx.systems], torch.complex128)
    est = None
    if est_out is not None:
        if est_out.dtype != torch.float64 or not est_out.is_cuda or tuple(est_out.shape) != (ctx.nsys, 4):
            raise ValueError("est_out must be a float64 CUDA tensor of shape (nsys, 4)")
        est = est_out.data_ptr()
    fresh = fresh or not ctx.stepping(walkers)
    flags = (STEP_REORTHO if reortho else 0) | (STEP_FRESH if fresh else 0)
    _check(load_library().afqmc_step(ctx.handle, w, xs, es, est, flags, _stream_handle(stream)))


def reorthogonalize(ctx: Context, walkers, stream=None):
    """afqmc_reorthogonalize: modified Gram-Schmidt of every walker's spin blocks."""
    _check(load_library().afqmc_reorthogonalize(ctx.handle, _walker_array(ctx, walkers), _stream_handle(stream)))


def overlap(ctx: Context, walkers, stream=None):
    """afqmc_overlap: log<Psi_T|phi> into walkers.log_ovlp."""
    _check(load_library().afqmc_overlap(ctx.handle, _walker_array(ctx, walkers), _stream_handle(stream)))


def greens_function(ctx: Context, walkers, theta_out, stream=None):
    """afqmc_greens_function: Theta = phi (Psi^T phi)^-1, complex128 [W, M, Nt] per system."""
    import torch
    w = _walker_array(ctx, walkers)
    th = _ptr_array(ctx, theta_out, [(s.nwalkers, s.nbasis, s.nalpha + s.nbeta) for s in ctx.systems],
                    torch.complex128)
    _check(load_library().afqmc_greens_function(ctx.handle, w, th, _stream_handle(stream)))


def force_bias(ctx: Context, walkers, vbias_out, stream=None):
    """afqmc_force_bias: vbias complex128 [W, G] per system."""
    import torch
    w = _walker_array(ctx, walkers)
    vb = _ptr_array(ctx, vbias_out, [(s.nwalkers, s.nchol) for s in ctx.systems], torch.complex128)
    _check(load_library().afqmc_force_bias(ctx.handle, w, vb, _stream_handle(stream)))


def get_info(ctx: Context, isys: int = 0) -> Info:
    info = Info()
    _check(load_library().afqmc_get_info(ctx.handle, isys, ctypes.byref(info)))
    return info


def set_timing(ctx: Context, enable: bool = True):
    """afqmc_set_timing: start (and zero) or stop the per-phase HIP-event timers."""
    _check(load_library().afqmc_set_timing(ctx.handle, 1 if enable else 0))


def get_timings(ctx: Context) -> dict:
    """afqmc_get_timings: {phase: (total ms, launches)} since timing was enabled."""
    t = Timings()
    _check(load_library().afqmc_get_timings(ctx.handle, ctypes.byref(t)))
    return {name: (t.ms[i], t.count[i]) for i, name in enumerate(PHASES)}


def destroy(ctx: Context):
    ctx.close()


def population_control(ctx: Context, walkers, u, parents_out=None, stream=None):
    """afqmc_population_control: comb resampling; u float64 [1] per system (device), in [0, 1)."""
    import torch
    w = _walker_array(ctx, walkers)
    us = _ptr_array(ctx, u, [(1,)] * ctx.nsys, torch.float64)
    ps = None
    if parents_out is not None:
        ps = _ptr_array(ctx, parents_out, [(s.nwalkers,) for s in ctx.systems], torch.int32)
    _check(load_library().afqmc_population_control(ctx.handle, w, us, ps, _stream_handle(stream)))


def set_e_shift(ctx: Context, e_shift: float, isys: int = 0, stream=None):
    """afqmc_set_e_shift: the energy shift E_T of the weight update (enqueued on the stream)."""
    _check(load_library().afqmc_set_e_shift(ctx.handle, isys, float(e_shift), _stream_handle(stream)))


def run_block(ctx: Context, walkers, x, e_out, est, u=None, step0: int = 0, reortho_every: int = 5,
              feedback: bool = True, fresh: bool = False, stream=None):
    """afqmc_run_block: nsteps walker steps with one estimator record each
    (est float64 [nsteps, 4] per system), then a comb with offset u (float64 [1]
    per system, or None for none) and, with `feedback`, E_T <- the block's
    estimate.  x: float64 [nsteps, W, G] per system; e_out complex128 [W, 3]."""
    import torch
    xs_list = x if isinstance(x, (list, tuple)) else [x]
    nsteps = int(xs_list[0].shape[0])
    w = _walker_array(ctx, walkers)
    xs = _ptr_array(ctx, xs_list, [(nsteps, s.nwalkers, s.nchol) for s in ctx.systems], torch.float64)
    es = _ptr_array(ctx, e_out, [(s.nwalkers, 3) for s in ctx.systems], torch.complex128)
    ests = _ptr_array(ctx, est, [(nsteps, 4)] * ctx.nsys, torch.float64)
    us = None if u is None else _ptr_array(ctx, u, [(1,)] * ctx.nsys, torch.float64)
    fresh = fresh or not ctx.stepping(walkers)
    flags = (BLOCK_FEEDBACK if feedback else 0) | (STEP_FRESH if fresh else 0)
    _check(load_library().afqmc_run_block(ctx.handle, w, xs, nsteps, int(step0), int(reortho_every), es, ests, us,
                                          flags, _stream_handle(stream)))


def reblock(series) -> dict:
    """afqmc_reblock (host): mean, the error bar at the chosen level (None when
    no level qualifies) and every level's (count, mean, std_err, std_err_err)."""
    x = np.ascontiguousarray(np.asarray(series, dtype=np.float64).ravel())
    r = ReblockResult()
    _check(load_library().afqmc_reblock(x.ctypes.data, int(x.size), ctypes.byref(r)))
    levels = [{"level": l, "n": int(r.count[l]), "mean": float(r.level_mean[l]), "std_err": float(r.std_err[l]),
               "std_err_err": float(r.std_err_err[l])} for l in range(r.nlevels)]
    opt = None if r.optimal < 0 else int(r.optimal)
    return {"n": int(r.n), "mean": float(r.mean), "optimal": opt,
            "std_err": levels[opt]["std_err"] if opt is not None else None, "levels": levels}


# ---- free projection --------------------------------------------------------------------

def _free_est(ctx: Context, est_out):
    import torch
    if est_out is None:
        return None
    if est_out.dtype != torch.float64 or not est_out.is_cuda or not est_out.is_contiguous() \
            or tuple(est_out.shape) != (ctx.nsys, FREE_EST):
        raise ValueError(f"est_out must be a contiguous float64 CUDA tensor of shape ({ctx.nsys}, {FREE_EST})")
    return est_out.data_ptr()


def free_propagate(ctx: Context, walkers, x, log_amp, stream=None):
    """afqmc_free_propagate: one free-projection step; x float64 [W, G], log_amp
    complex128 [W] (log of c <Psi_T|phi>, updated in place) per system."""
    import torch
    w = _walker_array(ctx, walkers)
    xs = _ptr_array(ctx, x, [(s.nwalkers, s.nchol) for s in ctx.systems], torch.float64)
    am = _ptr_array(ctx, log_amp, [(s.nwalkers,) for s in ctx.systems], torch.complex128)
    _check(load_library().afqmc_free_propagate(ctx.handle, w, xs, am, _stream_handle(stream)))


def free_estimator(ctx: Context, walkers, log_amp, e_in, est_out, stream=None):
    """afqmc_free_estimator: est_out float64 [nsys, 10] = (N, D, N1, N2 as
    re/im pairs, r, n); E(tau) = N / D."""
    import torch
    w = _walker_array(ctx, walkers)
    am = _ptr_array(ctx, log_amp, [(s.nwalkers,) for s in ctx.systems], torch.complex128)
    es = _ptr_array(ctx, e_in, [(s.nwalkers, 3) for s in ctx.systems], torch.complex128)
    _check(load_library().afqmc_free_estimator(ctx.handle, w, am, es, _free_est(ctx, est_out),
                                               _stream_handle(stream)))


def free_step(ctx: Context, walkers, x, log_amp, e_out, est_out=None, reortho=False, stream=None):
    """afqmc_free_step: free propagation, optional re-orthogonalisation, local
    energy and (with est_out) the free-projection estimate."""
    import torch
    w = _walker_array(ctx, walkers)
    xs = _ptr_array(ctx, x, [(s.nwalkers, s.nchol) for s in ctx.systems], torch.float64)
    am = _ptr_array(ctx, log_amp, [(s.nwalkers,) for s in ctx.systems], torch.complex128)
    es = _ptr_array(ctx, e_out, [(s.nwalkers, 3) for s in ctx.systems], torch.complex128)
    _check(load_library().afqmc_free_step(ctx.handle, w, xs, am, es, _free_est(ctx, est_out),
                                          STEP_REORTHO if reortho else 0, _stream_handle(stream)))


def free_energy(est_row) -> complex:
    """E(tau) = N / D from one row of a free-projection estimate."""
    r = [float(v) for v in est_row]
    return complex(r[0], r[1]) / complex(r[2], r[3])


# ---- learned control variate ---------------------------------------------------------

def _dev(t, dtype, shape, what):
    if t.dtype != dtype or not t.is_cuda or not t.is_contiguous() or tuple(t.shape) != tuple(shape):
        raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor of shape {tuple(shape)}")
    return t.data_ptr()


def cv_collect(ctx: Context, walkers, feat_out, ek_out, stream=None):
    """afqmc_cv_collect: features float64 [W, CV_NFEAT] and exact exchange complex128 [W] per system."""
    import torch
    w = _walker_array(ctx, walkers)
    fs = _ptr_array(ctx, feat_out, [(s.nwalkers, CV_NFEAT) for s in ctx.systems], torch.float64)
    es = _ptr_array(ctx, ek_out, [(s.nwalkers,) for s in ctx.systems], torch.complex128)
    _check(load_library().afqmc_cv_collect(ctx.handle, w, fs, es, _stream_handle(stream)))


def cv_train(ctx: Context, feat, ek, epochs: int, batch: int, lr: float, isys: int = 0, stream=None):
    """afqmc_cv_train (synchronous); returns the mean loss of each pass (float64 [epochs], on the GPU)."""
    import torch
    n = feat.shape[0]
    f = _dev(feat, torch.float64, (n, CV_NFEAT), "feat")
    e = _dev(ek, torch.complex128, (n,), "ek")
    loss = torch.zeros(max(1, epochs), dtype=torch.float64, device=feat.device)
    _check(load_library().afqmc_cv_train(ctx.handle, isys, f, e, n, epochs, batch, lr, loss.data_ptr(),
                                         _stream_handle(stream)))
    return loss[:epochs]


def cv_train_noalloc(ctx: Context, feat, ek, epochs: int, batch: int, lr: float, loss_out=None, isys: int = 0,
                     stream=None):
    """afqmc_cv_train_noalloc: the training of cv_train with the library's fixed
    workspace (no allocation, no synchronisation); loss_out: None or float64
    [epochs] on the GPU, filled with the mean loss of each pass."""
    import torch
    n = feat.shape[0]
    f = _dev(feat, torch.float64, (n, CV_NFEAT), "feat")
    e = _dev(ek, torch.complex128, (n,), "ek")
    lo = _dev(loss_out, torch.float64, (epochs,), "loss_out") if loss_out is not None else None
    _check(load_library().afqmc_cv_train_noalloc(ctx.handle, isys, f, e, n, epochs, batch, lr, lo,
                                                 _stream_handle(stream)))


def cv_set_params(ctx: Context, params=None, norm=None, isys: int = 0, stream=None):
    """afqmc_cv_set_params: params float32 [CV_NPARAMS] and/or norm float64 [CV_NNORM] (device)."""
    import torch
    p = _dev(params, torch.float32, (CV_NPARAMS,), "params") if params is not None else None
    q = _dev(norm, torch.float64, (CV_NNORM,), "norm") if norm is not None else None
    _check(load_library().afqmc_cv_set_params(ctx.handle, isys, p, q, _stream_handle(stream)))


def cv_get_params(ctx: Context, isys: int = 0, stream=None):
    """afqmc_cv_get_params: (params float32 [CV_NPARAMS], norm float64 [CV_NNORM]) on the GPU."""
    import torch
    params = torch.empty(CV_NPARAMS, dtype=torch.float32, device="cuda")
    norm = torch.empty(CV_NNORM, dtype=torch.float64, device="cuda")
    _check(load_library().afqmc_cv_get_params(ctx.handle, isys, params.data_ptr(), norm.data_ptr(),
                                              _stream_handle(stream)))
    return params, norm


def cv_predict(ctx: Context, feat, isys: int = 0, stream=None):
    """afqmc_cv_predict: predicted exchange energies (complex128 [n]) for raw features float64 [n, CV_NFEAT]."""
    import torch
    n = feat.shape[0]
    f = _dev(feat, torch.float64, (n, CV_NFEAT), "feat")
    out = torch.empty(n, dtype=torch.complex128, device=feat.device)
    _check(load_library().afqmc_cv_predict(ctx.handle, isys, f, n, out.data_ptr(), _stream_handle(stream)))
    return out


def cv_loss_grad(ctx: Context, x, t, isys: int = 0, stream=None):
    """afqmc_cv_loss_grad (synchronous): (loss float64 [1], gradient float32 [CV_NPARAMS]) on the GPU."""
    import torch
    n = x.shape[0]
    xp = _dev(x, torch.float32, (n, CV_NFEAT), "x")
    tp = _dev(t, torch.float32, (n, 2), "t")
    grad = torch.empty(CV_NPARAMS, dtype=torch.float32, device=x.device)
    loss = torch.empty(1, dtype=torch.float64, device=x.device)
    _check(load_library().afqmc_cv_loss_grad(ctx.handle, isys, xp, tp, n, grad.data_ptr(), loss.data_ptr(),
                                             _stream_handle(stream)))
    return loss, grad


def cv_state(ctx: Context, isys: int = 0, stream=None):
    """afqmc_cv_state: (predictions complex128 [W], subset int32 [k], call index int64 [1]) of the last energy call."""
    import torch
    s = ctx.systems[isys]
    k = get_info(ctx, isys).cv_subset
    f = torch.empty(s.nwalkers, dtype=torch.complex128, device="cuda")
    sub = torch.empty(max(1, k), dtype=torch.int32, device="cuda")
    call = torch.empty(1, dtype=torch.int64, device="cuda")
    _check(load_library().afqmc_cv_state(ctx.handle, isys, f.data_ptr(), sub.data_ptr() if k else None,
                                         call.data_ptr(), _stream_handle(stream)))
    return f, sub[:k], call

