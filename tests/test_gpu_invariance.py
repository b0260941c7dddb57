"""Bitwise invariances of the HIP path (no oracle needed: both sides run the
same kernels on the same inputs).

* Walker permutation: permuting the walkers (and their fields) permutes every
  per-walker output bit for bit — no walker's arithmetic depends on which other
  walkers share its launch tiles.
* Resume: 12 steps, a copy of the walker state through host memory into a new
  context, 8 more steps equal 20 uninterrupted steps bit for bit (the state a
  run needs is the caller-owned walker slab, weights, log-overlaps and flags).
"""
import numpy as np
import pytest

import afqmc_inputs as gi

pytestmark = pytest.mark.gpu

SPEC = gi.SystemSpec(100, 10, 9, 200, tau=75.0, seed=11)
W = 37


def _lib():
    import torch
    from paper_2406_16238_amd import afqmc as A
    return A, torch


def _setup(A, precision=0):
    h1, chol, ecore, trial = gi.make_system(SPEC)
    ctx = A.setup_hamiltonian(A.SystemInput(h1, chol, ecore, trial, SPEC.nalpha, SPEC.nbeta, W, 0.005),
                              A.default_options(precision=precision))
    return ctx, trial


def _host(w, e):
    return [w.phi.cpu().numpy(), w.weight.cpu().numpy(), w.log_ovlp.cpu().numpy(), w.flags.cpu().numpy(),
            e.cpu().numpy()]


@pytest.mark.parametrize("precision", [0, 3], ids=["fp64", "bf16x2"])
def test_walker_permutation(precision):
    A, torch = _lib()
    ctx, trial = _setup(A, precision)
    try:
        phis = gi.initial_walkers(trial, W, noise=0.05, seed=12)
        perm = np.random.default_rng(4).permutation(W)
        fs = gi.FieldStream(9, W, SPEC.nchol)
        xs = [fs.next() for _ in range(6)]
        outs = []
        for order in (np.arange(W), perm):
            w = A.Walkers.from_numpy(phis[order])
            A.overlap(ctx, w)
            e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            for k, x in enumerate(xs, start=1):
                A.step(ctx, w, torch.as_tensor(x[order], device="cuda"), e, reortho=(k == 5))
            torch.cuda.synchronize()
            outs.append(_host(w, e))
        for a, b, name in zip(outs[0], outs[1], ("phi", "weight", "log_ovlp", "flags", "energies")):
            assert np.ascontiguousarray(a[perm]).tobytes() == np.ascontiguousarray(b).tobytes(), name
    finally:
        ctx.close()


def test_resume_through_host_memory():
    A, torch = _lib()
    fs = gi.FieldStream(21, W, SPEC.nchol)
    xs = [torch.as_tensor(fs.next(), device="cuda") for _ in range(20)]
    ctx, trial = _setup(A)
    phis = gi.initial_walkers(trial, W, noise=0.02, seed=13)
    try:
        w = A.Walkers.from_numpy(phis)
        A.overlap(ctx, w)
        e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        saved = None
        for k in range(1, 21):
            A.step(ctx, w, xs[k - 1], e, reortho=(k % 5 == 0))
            if k == 12:
                torch.cuda.synchronize()
                saved = [t.cpu().numpy().copy() for t in (w.phi, w.weight, w.log_ovlp, w.flags)]
        torch.cuda.synchronize()
        straight = _host(w, e)
    finally:
        ctx.close()
    ctx2, _ = _setup(A)
    try:
        w2 = A.Walkers(*[torch.as_tensor(a, device="cuda") for a in saved])
        e2 = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        for k in range(13, 21):
            A.step(ctx2, w2, xs[k - 1], e2, reortho=(k % 5 == 0))
        torch.cuda.synchronize()
        resumed = _host(w2, e2)
    finally:
        ctx2.close()
    for a, b, name in zip(straight, resumed, ("phi", "weight", "log_ovlp", "flags", "energies")):
        assert a.tobytes() == b.tobytes(), name


def test_packed_cholesky_vhs_is_bitwise_the_full_product():
    """V_HS from the packed upper triangles of the L^g (and its symmetric
    unpacking) equals the product over the full matrices bit for bit."""
    A, torch = _lib()
    h1, chol, ecore, trial = gi.make_system(SPEC)
    outs = []
    for bits in (0, 8):
        o = A.default_options()
        o.reserved[0] = bits
        ctx = A.setup_hamiltonian(A.SystemInput(h1, chol, ecore, trial, SPEC.nalpha, SPEC.nbeta, W, 0.005), o)
        try:
            w = A.Walkers.from_numpy(gi.initial_walkers(trial, W, noise=0.05, seed=3))
            A.overlap(ctx, w)
            e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            fs = gi.FieldStream(2, W, SPEC.nchol)
            for k in range(1, 7):
                A.step(ctx, w, torch.as_tensor(fs.next(), device="cuda"), e, reortho=(k == 5))
            torch.cuda.synchronize()
            outs.append(_host(w, e))
        finally:
            ctx.close()
    for a, b, name in zip(outs[0], outs[1], ("phi", "weight", "log_ovlp", "flags", "energies")):
        assert a.tobytes() == b.tobytes(), name


def test_device_generated_cholesky_equals_host_twin():
    """chol_gen = 1 (the library draws the counter recipe's L on the device)
    gives the same trajectory, bit for bit, as the host-drawn twin array."""
    A, torch = _lib()
    spec = gi.SystemSpec(60, 6, 5, 240, tau=45.0, seed=5, recipe="counter")
    Wg = 24
    h1, chol, ecore, trial = gi.make_system(spec)
    gen = A.CholGen(spec.nchol, spec.seed, spec.tau, spec.scale_factor())
    outs = []
    for src in (chol, gen):
        ctx = A.setup_hamiltonian(A.SystemInput(h1, src, ecore, trial, spec.nalpha, spec.nbeta, Wg, 0.005))
        try:
            info = A.get_info(ctx, 0)
            w = A.Walkers.from_numpy(gi.initial_walkers(trial, Wg, noise=0.05, seed=6))
            A.overlap(ctx, w)
            e = torch.empty((Wg, 3), dtype=torch.complex128, device="cuda")
            fs = gi.FieldStream(8, Wg, spec.nchol)
            for k in range(1, 7):
                A.step(ctx, w, torch.as_tensor(fs.next(), device="cuda"), e, reortho=(k == 5))
            torch.cuda.synchronize()
            outs.append(_host(w, e) + [np.array([info.e_hf, info.const_c])])
        finally:
            ctx.close()
    for a, b, name in zip(outs[0], outs[1], ("phi", "weight", "log_ovlp", "flags", "energies", "scalars")):
        assert a.tobytes() == b.tobytes(), name
