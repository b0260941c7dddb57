"""Learned control variate of the exchange energy, through the C ABI.

Against the oracle (oracle/cv_oracle.py, pinned on the CPU): features and exact
exchange energies of walkers (1e-10 relative, FP64), the network's forward
pass, loss gradient and Adam training (FP32 on the device against float64:
FP32 tolerances), the subset draw (bit-exact walker indices), and each energy
call's per-walker Horvitz-Thompson estimate given its predictions and subset
(1e-10).  Statistically: the estimator is unbiased at fixed walkers, and a
trained network leaves less than a fifth of the variance a constant control
variate (the training mean of EK) leaves, and far less than plain subsampling.
"""
import math

import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from oracle import cv_oracle as CV
from pairs import Pair

pytestmark = pytest.mark.gpu


def cv_ctx(p, **kw):
    A = p.A
    o = A.default_options(ex_mode=A.EX_CV, **kw)
    return A.setup_hamiltonian(A.SystemInput(p.h1, p.chol, p.ecore, p.trial, p.spec.nalpha, p.spec.nbeta, p.W,
                                             p.dt), o)


def collect(p, ctx, phis):
    A, torch = p.A, p.torch
    w = A.Walkers.from_numpy(phis)
    feat = torch.empty((p.W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
    ek = torch.empty(p.W, dtype=torch.complex128, device="cuda")
    A.cv_collect(ctx, w, feat, ek)
    torch.cuda.synchronize()
    return feat, ek


@pytest.mark.parametrize("spec,W", [(gi.SMALL.system, 10), (gi.SystemSpec(100, 10, 9, 200, tau=75.0, seed=11), 37)],
                         ids=["small", "tiled-open-shell"])
def test_features_and_exchange_match_oracle(spec, W):
    p = Pair(spec, W, 0.005)
    try:
        phis = gi.initial_walkers(p.trial, W, noise=0.05, seed=8)
        feat, ek = collect(p, p.ctx, phis)
        feat, ek = feat.cpu().numpy(), ek.cpu().numpy()
        for k in np.unique(np.linspace(0, W - 1, 5).astype(int)):
            of = CV.features(p.ham, phis[k], O)
            oe = CV.exchange_energy(p.ham, phis[k], O)
            assert np.max(np.abs(feat[k] - of) / np.maximum(1.0, np.abs(of))) < 1e-10, k
            assert abs(ek[k] - oe) / max(1.0, abs(oe)) < 1e-10, k
    finally:
        p.close()


def _params64(A, ctx):
    params, norm = A.cv_get_params(ctx)
    return CV.unflatten(params.cpu().numpy().astype(np.float64)), norm.cpu().numpy()


def test_network_forward_and_gradient_match_oracle():
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        prm, norm = _params64(A, p.ctx)
        nf = A.CV_NFEAT
        assert np.allclose(norm, [0] * nf + [1] * nf + [0, 0, 1, 1])   # identity at set-up
        rng = np.random.default_rng(5)
        n = 37                                                        # ragged over 16-sample workgroups
        X = rng.standard_normal((n, A.CV_NFEAT)).astype(np.float32)
        T = rng.standard_normal((n, 2)).astype(np.float32)
        y, _ = CV.forward(prm, X.astype(np.float64))
        f = A.cv_predict(p.ctx, torch.as_tensor(X.astype(np.float64), device="cuda")).cpu().numpy()
        assert np.max(np.abs(f.real - y[:, 0])) < 1e-5 * max(1.0, np.abs(y).max())
        assert np.max(np.abs(f.imag - y[:, 1])) < 1e-5 * max(1.0, np.abs(y).max())
        loss, grad = A.cv_loss_grad(p.ctx, torch.as_tensor(X, device="cuda"), torch.as_tensor(T, device="cuda"))
        ol, og = CV.loss_and_grad(prm, X.astype(np.float64), T.astype(np.float64))
        assert abs(loss.item() - ol) < 1e-5 * ol
        og = CV.flatten(og)
        g = grad.cpu().numpy().astype(np.float64)
        assert np.max(np.abs(g - og)) < 1e-4 * np.abs(og).max()
    finally:
        p.close()


def test_training_matches_oracle_adam():
    """Normalisation from the samples, then Adam over minibatches, against the
    float64 oracle started from the same parameters."""
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        rng = np.random.default_rng(2)
        n, epochs, batch, lr = 100, 3, 32, 2e-3
        nf = A.CV_NFEAT
        feat = rng.standard_normal((n, nf)) * np.arange(1, nf + 1) + np.arange(nf)
        ek = feat[:, 0] * 0.3 - 0.1 * feat[:, 4] + 1j * (0.01 * feat[:, 1])
        start = CV.init_params(seed=9)
        A.cv_set_params(p.ctx, torch.as_tensor(CV.flatten(start).astype(np.float32), device="cuda"))
        losses = A.cv_train(p.ctx, torch.as_tensor(feat, device="cuda"), torch.as_tensor(ek, device="cuda"),
                            epochs, batch, lr).cpu().numpy()
        got, norm = _params64(A, p.ctx)
        # oracle: the same normalisation, minibatches and Adam in float64
        mu, sd = feat.mean(0), feat.std(0)
        tm = np.array([ek.real.mean(), ek.imag.mean()])
        ts = np.array([ek.real.std(), ek.imag.std()])
        assert np.allclose(norm, np.concatenate([mu, sd, tm, ts]), rtol=1e-12, atol=1e-14)
        X = (feat - mu) / sd
        T = (np.stack([ek.real, ek.imag], 1) - tm) / ts
        prm = {k: v.astype(np.float32).astype(np.float64) for k, v in start.items()}
        m = {k: np.zeros_like(v) for k, v in prm.items()}
        v = {k: np.zeros_like(x) for k, x in prm.items()}
        t, ol = 0, []
        for _ in range(epochs):
            tot = 0.0
            for b0 in range(0, n, batch):
                xb, tb = X[b0:b0 + batch], T[b0:b0 + batch]
                loss, g = CV.loss_and_grad(prm, xb, tb)
                tot += loss * len(xb) / n
                t += 1
                CV.adam_step(prm, g, m, v, t, lr)
            ol.append(tot)
        assert np.allclose(losses, ol, rtol=1e-4)
        a, b = CV.flatten(got), CV.flatten(prm)
        assert np.max(np.abs(a - b)) < 1e-4 * np.abs(b).max()
    finally:
        p.close()


def test_energy_call_is_the_horvitz_thompson_estimate():
    spec = gi.SystemSpec(100, 10, 9, 200, tau=75.0, seed=11)
    W = 40
    p = Pair(spec, W, 0.005)
    A, torch = p.A, p.torch
    ctx = cv_ctx(p, cv_seed=7)
    try:
        k = A.get_info(ctx, 0).cv_subset
        assert k == math.ceil(W / 8)
        # a rough network, so that f differs from EK
        phis = gi.initial_walkers(p.trial, W, noise=0.05, seed=21)
        feat, ek = collect(p, ctx, phis)
        A.cv_train(ctx, feat, ek, 5, 16, 1e-2)
        w = A.Walkers.from_numpy(phis)
        e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        for call in range(3):
            A.local_energy(ctx, w, e)
            f, sub, c = A.cv_state(ctx)
            torch.cuda.synchronize()
            assert c.item() == call
            S = CV.subset(7, call, W, k)
            assert np.array_equal(sub.cpu().numpy(), S)
            fw = f.cpu().numpy()
            # predictions are the network's on this call's features
            assert np.allclose(fw, A.cv_predict(ctx, feat).cpu().numpy(), rtol=0, atol=1e-12)
            ee = e.cpu().numpy()
            eks = np.array([CV.exchange_energy(p.ham, phis[j], O) for j in range(W)])
            g = CV.ht_exchange(fw, eks, S, k / W)
            for j in range(W):
                _, e1, e2 = O.local_energy(p.ham, phis[j])
                ej = e2 - eks[j]
                assert abs(ee[j, 1] - e1) < 1e-10 * max(1.0, abs(e1))
                assert abs(ee[j, 2] - (ej + g[j])) < 1e-10 * max(1.0, abs(e2)), (call, j)
                assert abs(ee[j, 0] - (e1 + ej + g[j])) < 1e-10 * max(1.0, abs(e1))
    finally:
        ctx.close()
        p.close()


def test_cv_trajectory_leaves_the_walkers_unchanged():
    """The control variate changes energies only: weights, overlaps and walkers
    of a trajectory equal those of the full-exchange path."""
    spec = gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11)
    p = Pair(spec, 48, 0.005)
    A, torch = p.A, p.torch
    ctx = cv_ctx(p)
    try:
        outs = []
        for c in (p.ctx, ctx):
            w = A.Walkers.from_numpy(gi.initial_walkers(p.trial, 48))
            A.overlap(c, w)
            e = torch.empty((48, 3), dtype=torch.complex128, device="cuda")
            fl = gi.FieldStream(3, 48, spec.nchol)
            for step in range(1, 8):
                A.step(c, w, torch.as_tensor(fl.next(), device="cuda"), e, reortho=(step % 5 == 0))
            torch.cuda.synchronize()
            outs.append((w.weight.cpu().numpy(), w.phi.cpu().numpy(), e.cpu().numpy()))
        (w0, f0, e0), (w1, f1, e1) = outs
        assert np.max(np.abs(w1 - w0) / np.abs(w0)) < 1e-10
        assert np.max(np.abs(f1 - f0)) < 1e-10 * np.abs(f0).max()
        assert np.max(np.abs(e1[:, 1] - e0[:, 1])) < 1e-10 * np.abs(e0[:, 1]).max()   # E1 untouched
    finally:
        ctx.close()
        p.close()


@pytest.mark.parametrize("precision", [0, 3], ids=["fp64", "bf16x2"])
def test_unbiased_and_variance_gain(precision):
    """At fixed walkers: the mean over many subset draws of the CV estimate of
    sum_w omega_w EK_w agrees with the exact value within its statistical error,
    and a trained network has a far smaller spread than plain subsampling."""
    spec = gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11)
    W = 128
    p = Pair(spec, W, 0.005)
    A, torch = p.A, p.torch
    ctx = cv_ctx(p, precision=precision)
    try:
        # training samples from a short trajectory of the CV context itself
        w = A.Walkers.from_numpy(gi.initial_walkers(p.trial, W, noise=0.02, seed=4))
        A.overlap(ctx, w)
        e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        fl = gi.FieldStream(5, W, spec.nchol)
        feats, eks = [], []
        for step in range(1, 31):
            A.step(ctx, w, torch.as_tensor(fl.next(), device="cuda"), e, reortho=(step % 5 == 0))
            f = torch.empty((W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
            k_ = torch.empty(W, dtype=torch.complex128, device="cuda")
            A.cv_collect(ctx, w, f, k_)
            feats.append(f)
            eks.append(k_)
        feat, ek = torch.cat(feats), torch.cat(eks)
        losses = A.cv_train(ctx, feat, ek, 40, 128, 2e-3).cpu().numpy()
        print(f"training loss {losses[0]:.3e} -> {losses[-1]:.3e}")
        # fixed walkers: the last state
        wt = w.weight.cpu().numpy()
        om = wt / wt.sum()

        def draws(R):
            """sum_w omega_w Re E2_w over R energy calls (E2 = EJ + g, EJ fixed)."""
            vals = []
            for _ in range(R):
                A.local_energy(ctx, w, e)
                vals.append(np.sum(om * e.cpu().numpy()[:, 2].real))
            return np.array(vals)

        e2_cv = draws(200)
        full = A.setup_hamiltonian(A.SystemInput(p.h1, p.chol, p.ecore, p.trial, spec.nalpha, spec.nbeta, W, p.dt),
                                   A.default_options(precision=precision))
        try:
            e_full = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
            A.local_energy(full, w, e_full)
            exact_e2 = np.sum(om * e_full.cpu().numpy()[:, 2].real)
        finally:
            full.close()
        sd = e2_cv.std(ddof=1)
        print(f"CV: mean - exact {e2_cv.mean() - exact_e2:.3e} Ha, spread {sd:.3e} Ha")
        assert abs(e2_cv.mean() - exact_e2) < 4 * sd / math.sqrt(len(e2_cv)) + 1e-12
        # the method without the network: a constant control variate, the
        # training mean of EK (zero weights keep only the target normalisation)
        zp = torch.zeros(A.CV_NPARAMS, dtype=torch.float32, device="cuda")
        _, trained_norm = A.cv_get_params(ctx)
        A.cv_set_params(ctx, zp, trained_norm)
        e2_const = draws(200)
        sc = e2_const.std(ddof=1)
        print(f"constant mean: mean - exact {e2_const.mean() - exact_e2:.3e} Ha, spread {sc:.3e} Ha; "
              f"variance ratio network / constant {sd**2 / sc**2:.2e}")
        assert abs(e2_const.mean() - exact_e2) < 4 * sc / math.sqrt(len(e2_const))
        # plain subsampling: f = 0 (zero network, zero target mean)
        nf = A.CV_NFEAT
        zn = torch.tensor([0.0] * nf + [1.0] * nf + [0.0, 0.0, 1.0, 1.0], dtype=torch.float64, device="cuda")
        A.cv_set_params(ctx, zp, zn)
        e2_plain = draws(200)
        sp = e2_plain.std(ddof=1)
        print(f"plain subsampling: mean - exact {e2_plain.mean() - exact_e2:.3e} Ha, spread {sp:.3e} Ha; "
              f"variance ratio {sd**2 / sp**2:.2e}")
        assert abs(e2_plain.mean() - exact_e2) < 4 * sp / math.sqrt(len(e2_plain))
        # the trained network must remove most of what a constant leaves
        assert sd ** 2 < 0.2 * sc ** 2
        assert sd ** 2 < 0.01 * sp ** 2
    finally:
        ctx.close()
        p.close()


def test_cv_in_a_system_set():
    """Each system of a set has its own network and subset draws; the set's
    energies equal those of separate single-system contexts bit for bit."""
    from test_gpu_batching import small_set, make_inputs, assert_bitwise
    import torch
    from paper_2406_16238_amd import afqmc as A
    inputs = make_inputs(A, small_set(4))
    opts = dict(ex_mode=A.EX_CV)
    walkers = [gi.initial_walkers(t, s.nwalkers, noise=0.03, seed=50 + i) for i, (s, t) in enumerate(inputs)]

    together = A.setup_hamiltonian([s for s, _ in inputs], A.default_options(**opts))
    try:
        ws = [A.Walkers.from_numpy(p) for p in walkers]
        es = [torch.empty((s.nwalkers, 3), dtype=torch.complex128, device="cuda") for s, _ in inputs]
        for _ in range(2):
            A.local_energy(together, ws, es)
        torch.cuda.synchronize()
        got = [e.cpu().numpy() for e in es]
    finally:
        together.close()
    for i, (s, _) in enumerate(inputs):
        one = A.setup_hamiltonian(s, A.default_options(**opts))
        try:
            w = A.Walkers.from_numpy(walkers[i])
            e = torch.empty((s.nwalkers, 3), dtype=torch.complex128, device="cuda")
            for _ in range(2):
                A.local_energy(one, w, e)
            torch.cuda.synchronize()
            assert_bitwise({"e": e.cpu().numpy()}, {"e": got[i]}, f"system {i}")
        finally:
            one.close()
