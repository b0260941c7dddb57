"""The C ABI library loads, exports every declared entry point and rejects bad
arguments before touching the device (no GPU needed)."""
import ctypes
import math
import os
import re

import numpy as np
import pytest

from paper_2406_16238_amd import afqmc as A

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lib():
    if not os.path.exists(A.LIB_PATH):
        from paper_2406_16238_amd import build
        build.build()
    return A.load_library()


def declared_functions():
    text = open(os.path.join(ROOT, "include", "afqmc.h")).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(afqmc_[a-z_0-9]+)\s*\(", text)))


def test_every_declared_symbol_is_exported(lib):
    names = declared_functions()
    assert len(names) >= 14
    for n in names:
        assert hasattr(lib, n), n
    assert set(names) == set(A.EXPORTS)


def test_library_defines_every_kernel_it_launches(lib):
    """Every symbol of the library's own namespace that it references is
    defined in it: a kernel whose host launch stub went missing would only
    fail when the library is loaded on a machine with a GPU."""
    import shutil
    import subprocess
    nm = shutil.which("nm")
    if nm is None:
        pytest.skip("nm not available")
    out = subprocess.run([nm, "-D", "--undefined-only", A.LIB_PATH], capture_output=True, text=True, check=True).stdout
    missing = [ln.split()[-1] for ln in out.splitlines() if "_ZN5afqmc" in ln]
    assert not missing, missing


def test_default_options(lib):
    o = A.default_options()
    assert o.precision == A.FP64 and o.taylor_order == 6 and o.fb_cap == 1.0
    assert math.isnan(o.e_shift) and o.mem_limit_bytes == 0
    assert o.streams == 0 and o.use_graph == 0 and o.tune == 1 and o.ex_mode == A.EX_FULL
    assert o.cv_fraction == 0.125 and o.cv_seed == 7 and o.tune_cache is None and o.deterministic == 1
    assert list(o.reserved) == [0] * 8
    assert lib.afqmc_default_options(None) == A.ERR_ARG


def _desc(m=6, na=2, nb=2, g=4, w=3, dt=0.01):
    h1 = np.eye(m)
    chol = np.zeros((g, m, m))
    trial = np.zeros((m, na + nb))
    keep = (h1, chol, trial)
    d = A.SystemDesc(m, na, nb, g, w, h1.ctypes.data, chol.ctypes.data, 0.0, trial.ctypes.data, dt)
    return d, keep


@pytest.mark.parametrize("field,value,status", [
    ("nbasis", 0, A.ERR_ARG), ("nchol", -1, A.ERR_ARG), ("nwalkers", 0, A.ERR_ARG),
    ("nalpha", 7, A.ERR_ARG), ("dt", 0.0, A.ERR_ARG), ("dt", float("nan"), A.ERR_ARG),
    ("ecore", float("inf"), A.ERR_ARG), ("h1", None, A.ERR_ARG), ("trial", None, A.ERR_ARG),
    ("chol", None, A.ERR_ARG), ("chol_gen", 2, A.ERR_ARG),
])
def test_setup_rejects_bad_descriptions(lib, field, value, status):
    d, keep = _desc()
    setattr(d, field, value)
    out = ctypes.c_void_p(123)
    r = lib.afqmc_setup_hamiltonian(ctypes.byref(d), 1, None, None, ctypes.byref(out))
    assert r == status
    assert out.value is None
    assert len(A.last_error()) > 0


def test_setup_rejects_bad_generator(lib):
    for tau, scale in ((0.0, 1.0), (float("nan"), 1.0), (1.0, float("inf"))):
        d, keep = _desc()
        d.chol, d.chol_gen, d.gen_tau, d.gen_scale = None, 1, tau, scale
        out = ctypes.c_void_p()
        assert lib.afqmc_setup_hamiltonian(ctypes.byref(d), 1, None, None, ctypes.byref(out)) == A.ERR_ARG


def test_setup_rejects_wide_spin_blocks(lib):
    d, keep = _desc(m=80, na=60, nb=2)
    out = ctypes.c_void_p()
    assert lib.afqmc_setup_hamiltonian(ctypes.byref(d), 1, None, None, ctypes.byref(out)) == A.ERR_UNSUPPORTED


def test_setup_rejects_bad_options(lib):
    d, keep = _desc()
    out = ctypes.c_void_p()
    for field, value in (("taylor_order", 0), ("taylor_order", 17), ("precision", 9), ("fb_cap", float("nan")),
                         ("streams", -1), ("ex_mode", 2), ("cv_fraction", 0.0), ("cv_fraction", 1.5),
                         ("cv_fraction", float("nan")), ("prop_precision", 2), ("deterministic", 0),
                         ("deterministic", 2)):
        o = A.default_options()
        setattr(o, field, value)
        assert lib.afqmc_setup_hamiltonian(ctypes.byref(d), 1, ctypes.byref(o), None, ctypes.byref(out)) \
            == A.ERR_ARG, field
    assert lib.afqmc_setup_hamiltonian(ctypes.byref(d), 0, None, None, ctypes.byref(out)) == A.ERR_ARG
    assert lib.afqmc_setup_hamiltonian(None, 1, None, None, ctypes.byref(out)) == A.ERR_ARG
    assert lib.afqmc_setup_hamiltonian(ctypes.byref(d), 1, None, None, None) == A.ERR_ARG


def test_step_calls_reject_null_context(lib):
    w = A.CWalkers()
    assert lib.afqmc_propagate(None, ctypes.byref(w), None, None) == A.ERR_ARG
    assert lib.afqmc_local_energy(None, ctypes.byref(w), None, None, None) == A.ERR_ARG
    assert lib.afqmc_reorthogonalize(None, ctypes.byref(w), None) == A.ERR_ARG
    assert lib.afqmc_step(None, ctypes.byref(w), None, None, None, 0, None) == A.ERR_ARG
    assert lib.afqmc_overlap(None, None, None) == A.ERR_ARG
    assert lib.afqmc_greens_function(None, None, None, None) == A.ERR_ARG
    assert lib.afqmc_force_bias(None, None, None, None) == A.ERR_ARG
    info = A.Info()
    assert lib.afqmc_get_info(None, 0, ctypes.byref(info)) == A.ERR_ARG
    assert lib.afqmc_set_timing(None, 1) == A.ERR_ARG
    assert lib.afqmc_get_timings(None, None) == A.ERR_ARG
    assert lib.afqmc_cv_collect(None, None, None, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_train(None, 0, None, None, 10, 1, 1, 1e-3, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_set_params(None, 0, None, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_get_params(None, 0, None, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_predict(None, 0, None, 1, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_loss_grad(None, 0, None, None, 1, None, None, None) == A.ERR_ARG
    assert lib.afqmc_cv_state(None, 0, None, None, None, None) == A.ERR_ARG
    assert lib.afqmc_population_control(None, None, None, None, None) == A.ERR_ARG
    assert lib.afqmc_set_e_shift(None, 0, 0.0, None) == A.ERR_ARG
    assert lib.afqmc_run_block(None, ctypes.byref(w), None, 1, 0, 5, None, None, None, 0, None) == A.ERR_ARG
    assert lib.afqmc_free_propagate(None, ctypes.byref(w), None, None, None) == A.ERR_ARG
    assert lib.afqmc_free_estimator(None, ctypes.byref(w), None, None, None, None) == A.ERR_ARG
    assert lib.afqmc_free_step(None, ctypes.byref(w), None, None, None, None, 0, None) == A.ERR_ARG
    lib.afqmc_destroy(None)  # no-op


def test_struct_layouts_match_header(tmp_path):
    """ctypes layouts equal what a C compiler makes of include/afqmc.h."""
    import subprocess
    fields = {"afqmc_system_desc": (A.SystemDesc, ["nbasis", "nalpha", "nbeta", "nchol", "nwalkers", "h1", "chol",
                                                   "ecore", "trial", "dt", "chol_gen", "reserved_desc", "gen_seed",
                                                   "gen_tau", "gen_scale"]),
              "afqmc_options": (A.Options, ["precision", "taylor_order", "fb_cap", "e_shift", "mem_limit_bytes",
                                            "streams", "use_graph", "tune", "ex_mode", "cv_fraction", "cv_seed",
                                            "prop_precision", "deterministic", "tune_cache", "reserved"]),
              "afqmc_walkers": (A.CWalkers, ["phi", "weight", "log_ovlp", "flags"]),
              "afqmc_info": (A.Info, ["e_hf", "e_shift", "const_c", "device_bytes", "exchange_tile", "exchange_order", "lane",
                                      "graph_captures", "graph_replays", "cv_subset", "vhs_tile", "taylor_tile",
                                      "reserved_info"]),
              "afqmc_timings": (A.Timings, ["ms", "count"]),
              "afqmc_reblock_result": (A.ReblockResult, ["n", "mean", "nlevels", "optimal", "count", "level_mean",
                                                         "std_err", "std_err_err"])}
    lines = ['#include <stdio.h>', '#include <stddef.h>', '#include "afqmc.h"', "int main(void) {"]
    for cname, (_, fl) in fields.items():
        lines.append(f'printf("{cname} size %zu\\n", sizeof({cname}));')
        for f in fl:
            lines.append(f'printf("{cname} {f} %zu\\n", offsetof({cname}, {f}));')
    lines.append("return 0; }")
    src = tmp_path / "layout.c"
    src.write_text("\n".join(lines))
    exe = tmp_path / "layout"
    subprocess.run(["gcc", "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], capture_output=True, text=True, check=True).stdout.split("\n")
    got = {}
    for line in out:
        if line:
            a, b, c = line.split()
            got[(a, b)] = int(c)
    for cname, (cls, fl) in fields.items():
        assert got[(cname, "size")] == ctypes.sizeof(cls), cname
        for f in fl:
            assert got[(cname, f)] == getattr(cls, f).offset, (cname, f)
