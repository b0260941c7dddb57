"""Precision form: exchange and force bias in FP32, in split BF16 (three
bfloat16 terms and six products, or two terms and three products), or in one
FP16 / BF16 product of the walkers' departure from the trial with the trial's
part exact (the trial split); FP32 accumulation; overlaps, LU, propagation,
weights and re-orthogonalisation in FP64.

Bar: per-walker local energies within 0.1 mHa of the FP64 path (and of the
oracle) on identical walker states; the mixed estimator of a short trajectory
driven by the same fields within 0.1 mHa of the FP64 trajectory's.
"""
import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from pairs import Pair, cmp_rel

pytestmark = pytest.mark.gpu
MHA = 1e-3
FORMS = {"fp32": 1, "bf16x3": 2, "bf16x2": 3, "fp16t": 4, "bf16t": 5}


def ctx_for(p, precision):
    A = p.A
    return A.setup_hamiltonian(A.SystemInput(p.h1, p.chol, p.ecore, p.trial, p.spec.nalpha, p.spec.nbeta, p.W,
                                             p.dt), A.default_options(precision=precision))


def energies(p, ctx, phis):
    A, torch = p.A, p.torch
    w = A.Walkers.from_numpy(phis)
    A.overlap(ctx, w)
    e = torch.empty((p.W, 3), dtype=torch.complex128, device="cuda")
    A.local_energy(ctx, w, e)
    torch.cuda.synchronize()
    return e.cpu().numpy()


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("spec,W", [(gi.SMALL.system, 10), (gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11), 70),
                                    (gi.SystemSpec(96, 42, 41, 192, tau=70.0, seed=13), 9),
                                    (gi.HEADLINE.system, 256)], ids=["small", "tiled", "wide", "headline"])
def test_energy_error_on_identical_walkers(form, spec, W):
    p = Pair(spec, W, 0.005)
    ctx = ctx_for(p, FORMS[form])
    try:
        phis = gi.initial_walkers(p.trial, W, noise=0.02, seed=31)
        e64 = energies(p, p.ctx, phis)
        elp = energies(p, ctx, phis)
        err = np.abs(elp - e64)
        print(f"{form} M={spec.nbasis}: max |dE| {err[:, 0].max():.2e} Ha, rms {np.sqrt((err[:, 0]**2).mean()):.2e}")
        assert err.max() < 0.1 * MHA
        for k in np.unique(np.linspace(0, W - 1, 3).astype(int)):
            oe = np.array(O.local_energy(p.ham, phis[k]))
            assert np.abs(elp[k] - oe).max() < 0.1 * MHA
        # the reduced form is not silently the FP64 path
        assert err[:, 2].max() > 0.0
    finally:
        ctx.close()
        p.close()


@pytest.mark.parametrize("form", list(FORMS))
def test_force_bias_error(form):
    """vbias enters through the trace of the exchange matrices: check it by the
    Coulomb energy EJ = 1/2 sum vbias^2 of the FP32/BF16 path after a step."""
    spec = gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11)
    p = Pair(spec, 32, 0.005)
    ctx = ctx_for(p, FORMS[form])
    try:
        A, torch = p.A, p.torch
        phis = gi.initial_walkers(p.trial, 32, noise=0.02, seed=5)
        fields = gi.FieldStream(2, 32, spec.nchol)
        outs = []
        for c in (p.ctx, ctx):
            w = A.Walkers.from_numpy(phis)
            A.overlap(c, w)
            e = torch.empty((32, 3), dtype=torch.complex128, device="cuda")
            fl = gi.FieldStream(2, 32, spec.nchol)
            for step in range(4):
                A.step(c, w, torch.as_tensor(fl.next(), device="cuda"), e, reortho=(step == 2))
            torch.cuda.synchronize()
            outs.append((e.cpu().numpy(), w.weight.cpu().numpy(), w.phi.cpu().numpy()))
        (e64, w64, f64), (elp, wlp, flp) = outs
        assert np.abs(elp - e64).max() < 0.1 * MHA
        assert cmp_rel(wlp, w64) < 1e-4       # the force bias moved the weights only slightly
        assert cmp_rel(flp, f64, np.abs(f64).max()) < 1e-4
    finally:
        ctx.close()
        p.close()


@pytest.mark.parametrize("form", list(FORMS))
def test_mixed_estimator_of_a_trajectory(form):
    spec = gi.MEDIUM.system
    p = Pair(spec, 128, 0.005)
    ctx = ctx_for(p, FORMS[form])
    try:
        A, torch = p.A, p.torch
        res = []
        for c in (p.ctx, ctx):
            w = A.Walkers.from_numpy(gi.initial_walkers(p.trial, 128))
            A.overlap(c, w)
            e = torch.empty((128, 3), dtype=torch.complex128, device="cuda")
            est = torch.empty((1, 4), dtype=torch.float64, device="cuda")
            fl = gi.FieldStream(0, 128, spec.nchol)
            mixed = []
            for step in range(1, 11):
                A.step(c, w, torch.as_tensor(fl.next(), device="cuda"), e, est, reortho=(step % 5 == 0))
                h = est.cpu().numpy()[0]
                mixed.append(h[0] / h[1])
            res.append(np.array(mixed))
        d = np.abs(res[1] - res[0])
        print(f"{form}: mixed-estimator difference over 10 steps max {d.max():.2e} Ha")
        assert d.max() < 0.1 * MHA
    finally:
        ctx.close()
        p.close()


@pytest.mark.parametrize("form", ["fp16t", "bf16t"])
def test_trial_split_at_the_trial_is_exact_to_fp32(form):
    """Walkers equal to the trial (Q = 0): the split forms reduce to T = T0,
    set up once in FP32, so the energies match FP64 to FP32 rounding."""
    p = Pair(gi.SystemSpec(100, 10, 9, 200, tau=75.0, seed=11), 6, 0.005)
    ctx = ctx_for(p, FORMS[form])
    try:
        phis = gi.initial_walkers(p.trial, 6)
        err = np.abs(energies(p, ctx, phis) - energies(p, p.ctx, phis))
        assert err.max() < 1e-6
    finally:
        ctx.close()
        p.close()


@pytest.mark.parametrize("form", list(FORMS))
@pytest.mark.parametrize("spec,W", [(gi.SystemSpec(37, 5, 3, 70, tau=30.0, seed=7), 11),
                                    (gi.SystemSpec(18, 3, 2, 1, tau=5.0, seed=24), 7),
                                    (gi.SystemSpec(30, 4, 4, 6, tau=10.0, seed=27), 5)],
                         ids=["g70-open-shell", "one-vector", "g6"])
def test_cholesky_counts_off_the_workgroup_tile(form, spec, W):
    """Cholesky-vector counts that are no multiple of the four vectors a 16-bit
    exchange workgroup covers (so that the second vector of a wave can be a
    padded one), and odd walker counts: the padded vectors and walkers must add
    nothing.  Per-walker energies on identical walkers against the oracle, and
    a short trajectory (weights move by the force bias, i.e. vbias from the
    trace of the exchange) against the FP64 path on the same fields."""
    p = Pair(spec, W, 0.005)
    ctx = ctx_for(p, FORMS[form])
    try:
        A, torch = p.A, p.torch
        phis = gi.initial_walkers(p.trial, W, noise=0.02, seed=41)
        ref = O.local_energies(p.ham, phis)
        elp = energies(p, ctx, phis)
        assert np.abs(elp - ref).max() < 0.1 * MHA
        outs = []
        for c in (p.ctx, ctx):
            w = A.Walkers.from_numpy(phis)
            A.overlap(c, w)
            e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            fl = gi.FieldStream(3, W, spec.nchol)
            for step in range(3):
                A.step(c, w, torch.as_tensor(fl.next(), device="cuda"), e)
            torch.cuda.synchronize()
            outs.append((e.cpu().numpy(), w.weight.cpu().numpy()))
        (e64, w64), (e2, w2) = outs
        assert np.abs(e2 - e64).max() < 0.1 * MHA
        assert cmp_rel(w2, w64) < 1e-4
    finally:
        ctx.close()
        p.close()
