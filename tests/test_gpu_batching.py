"""Batching form: several independent systems in one context, spread over the
library's internal streams and optionally replayed from a hipGraph.

Bar: every walker quantity of every system is bitwise equal to what a
separate single-system context computes from the same inputs (all reductions
are deterministic and no kernel depends on which other systems share the
device).
"""
import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from pairs import cmp_rel

pytestmark = pytest.mark.gpu


def _lib():
    import torch
    from paper_2406_16238_amd import afqmc as A
    return A, torch


def small_set(n=16):
    """Sixteen uneven systems of the batching workload's shape (M = 10 N,
    Nchol = 4 M, walker counts from the same seeded draw), scaled down so that
    the test runs in seconds; one open-shell system among them."""
    counts = gi.batching_walker_counts()
    specs = []
    for k in range(n):
        m = 24 + 8 * k
        na = max(2, m // 10)
        nb = na - 1 if k == 5 else na
        specs.append((gi.SystemSpec(m, na, nb, 4 * m, tau=0.75 * m, seed=100 + k), max(8, counts[k] // 8)))
    return specs


def make_inputs(A, specs, dt=0.005):
    out = []
    for spec, W in specs:
        h1, chol, ecore, trial = gi.make_system(spec)
        out.append((A.SystemInput(h1, chol, ecore, trial, spec.nalpha, spec.nbeta, W, dt), trial))
    return out


def run_steps(A, torch, ctx, inputs, nsteps, sys_index=None, check_each=None):
    """Steps the walkers of `inputs` (all systems of ctx) with fields from fixed
    per-system streams; buffers keep their addresses across steps."""
    idx = list(range(len(inputs))) if sys_index is None else sys_index
    walkers, xbuf, ebuf, streams = [], [], [], []
    for j in idx:
        sysin, trial = inputs[j]
        walkers.append(A.Walkers.from_numpy(gi.initial_walkers(trial, sysin.nwalkers, seed=40 + j)))
        xbuf.append(torch.empty((sysin.nwalkers, sysin.nchol), dtype=torch.float64, device="cuda"))
        ebuf.append(torch.empty((sysin.nwalkers, 3), dtype=torch.complex128, device="cuda"))
        streams.append(gi.FieldStream(60 + j, sysin.nwalkers, sysin.nchol))
    est = torch.empty((len(idx), 4), dtype=torch.float64, device="cuda")
    A.overlap(ctx, walkers)
    for step in range(1, nsteps + 1):
        for xb, fs in zip(xbuf, streams):
            xb.copy_(torch.as_tensor(fs.next()))
        A.step(ctx, walkers, xbuf, ebuf, est, reortho=(step % 5 == 0))
        if check_each is not None:
            torch.cuda.synchronize()
            check_each(step, walkers, ebuf, est)
    torch.cuda.synchronize()
    return walkers, ebuf, est


def snapshot(walkers, ebuf, est, k):
    w = walkers[k]
    return {"phi": w.phi.cpu().numpy(), "weight": w.weight.cpu().numpy(), "log_ovlp": w.log_ovlp.cpu().numpy(),
            "flags": w.flags.cpu().numpy(), "e": ebuf[k].cpu().numpy(), "est": est[k].cpu().numpy()}


def assert_bitwise(a, b, what):
    for key in a:
        x, y = np.ascontiguousarray(a[key]), np.ascontiguousarray(b[key])
        assert x.shape == y.shape and x.tobytes() == y.tobytes(), f"{what}: {key} differs"


@pytest.mark.parametrize("precision", [0, 1], ids=["fp64", "fp32"])
@pytest.mark.parametrize("graph", [False, True], ids=["eager", "graph"])
def test_set_equals_separate_runs_bitwise(precision, graph):
    A, torch = _lib()
    specs = small_set()
    inputs = make_inputs(A, specs)
    nsteps = 7
    ctx = A.setup_hamiltonian([s for s, _ in inputs], A.default_options(precision=precision, streams=4,
                                                                        use_graph=int(graph)))
    try:
        lanes = {A.get_info(ctx, i).lane for i in range(len(inputs))}
        assert lanes == {0, 1, 2, 3}
        walkers, ebuf, est = run_steps(A, torch, ctx, inputs, nsteps)
        together = [snapshot(walkers, ebuf, est, k) for k in range(len(inputs))]
        if graph:
            info = A.get_info(ctx, 0)
            print(f"graph captures {info.graph_captures}, replays {info.graph_replays}")
            assert info.graph_replays >= nsteps - 3
    finally:
        ctx.close()
    # walker 0 of every system against the oracle, which steps it alone on the
    # same fields (walkers are independent without population control)
    for k, (spec, W) in enumerate(specs):
        sysin, trial = inputs[k]
        ham = O.build(sysin.h1, sysin.chol, sysin.ecore, trial, spec.nalpha, spec.nbeta, sysin.dt)
        phi = gi.initial_walkers(trial, W, seed=40 + k)[:1]
        fs = gi.FieldStream(60 + k, W, sysin.nchol)
        ow, ologo = np.ones(1), O.initial_logo(ham, phi)
        for step in range(1, nsteps + 1):
            phi, ow, ologo, _ = O.propagate(ham, phi, ow, ologo, fs.next()[:1])
            if step % 5 == 0:
                phi, ologo = O.reorthogonalize(ham, phi, ologo)
        oe = np.array(O.local_energy(ham, phi[0]))
        g = together[k]
        tol = 1e-10 if precision == 0 else 1e-5
        assert cmp_rel(g["e"][0], oe) < tol, k
        assert cmp_rel(g["weight"][:1], ow) < tol, k
        assert cmp_rel(g["phi"][0], phi[0], np.abs(phi[0]).max()) < tol, k
    for k in range(len(inputs)):
        one = A.setup_hamiltonian(inputs[k][0], A.default_options(precision=precision, streams=1))
        try:
            w1, e1, s1 = run_steps(A, torch, one, inputs, nsteps, sys_index=[k])
            assert_bitwise(snapshot(w1, e1, s1, 0), together[k], f"system {k}")
        finally:
            one.close()


def test_graph_replays_match_eager_each_step():
    """Replayed steps, with eager work and synchronisations between them, give
    the eager path's results bit for bit at every step."""
    A, torch = _lib()
    inputs = make_inputs(A, [(gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11), 70)])
    eager = A.setup_hamiltonian(inputs[0][0], A.default_options())
    graph = A.setup_hamiltonian(inputs[0][0], A.default_options(use_graph=1))
    try:
        ref = {}

        def keep(step, walkers, ebuf, est):
            ref[step] = snapshot(walkers, ebuf, est, 0)

        run_steps(A, torch, eager, inputs, 12, check_each=keep)

        def check(step, walkers, ebuf, est):
            # eager work of the program's own between replays
            junk = torch.randn(1000, device="cuda").sum()
            assert torch.isfinite(junk)
            assert_bitwise(snapshot(walkers, ebuf, est, 0), ref[step], f"step {step}")

        run_steps(A, torch, graph, inputs, 12, check_each=check)
        info = A.get_info(graph, 0)
        assert info.graph_captures <= 4 and info.graph_replays >= 8
    finally:
        eager.close()
        graph.close()


@pytest.mark.parametrize("precision", [0, 1, 2, 3, 4], ids=["fp64", "fp32", "bf16x3", "bf16x2", "fp16t"])
def test_exchange_launch_shape_does_not_change_results(precision):
    """Walker tiling (FP64 kernel) and tile order (all exchange kernels) are
    speed knobs only: results are bitwise equal for every choice."""
    A, torch = _lib()
    inputs = make_inputs(A, [(gi.SystemSpec(100, 10, 9, 200, tau=75.0, seed=11), 37)])
    outs = []
    shapes = [(1, 1), (2, 4), (4, 16), (2, 1), (2, 5)] if precision == 0 else [(2, 1), (2, 4), (2, 16), (2, 3)]
    for wx, order in shapes:
        o = A.default_options(precision=precision)
        o.reserved[1] = wx
        o.reserved[2] = order
        ctx = A.setup_hamiltonian(inputs[0][0], o)
        try:
            info = A.get_info(ctx, 0)
            assert info.exchange_tile == wx and info.exchange_order == (0 if order == 1 else order)
            walkers, ebuf, est = run_steps(A, torch, ctx, inputs, 3)
            outs.append(snapshot(walkers, ebuf, est, 0))
        finally:
            ctx.close()
    for k in range(1, len(outs)):
        assert_bitwise(outs[0], outs[k], f"launch shape {shapes[0]} vs {shapes[k]}")
