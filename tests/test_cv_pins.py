"""Pins of the control-variate oracle (CPU only)."""
import itertools

import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from oracle import cv_oracle as CV


def test_p16_horvitz_thompson_is_unbiased_and_has_the_stated_variance():
    """Exact expectation over all C(16, 2) subsets equals the full-exchange
    estimator; the spread over subsets equals the finite-population variance."""
    rng = np.random.default_rng(3)
    W, k = 16, 2
    pi = k / W
    weights = rng.uniform(0.5, 1.5, W)
    omega = weights / weights.sum()
    ek = rng.normal(-1.5, 0.05, W) + 1j * rng.normal(0, 0.01, W)
    f = ek + rng.normal(0, 0.02, W)          # an imperfect predictor
    full = np.sum(omega * ek)
    vals = []
    for S in itertools.combinations(range(W), k):
        g = CV.ht_exchange(f, ek, S, pi)
        vals.append(np.sum(omega * g))
    vals = np.array(vals)
    assert abs(vals.mean() - full) < 1e-14
    var = np.mean((vals.real - full.real) ** 2)
    assert abs(var - CV.cv_variance(omega, (ek - f).real, pi)) < 1e-12 * max(var, 1e-30) + 1e-18
    # and per walker: E_S[g_w] = EK_w
    g_all = np.array([CV.ht_exchange(f, ek, S, pi) for S in itertools.combinations(range(W), k)])
    assert np.max(np.abs(g_all.mean(0) - ek)) < 1e-13


def test_p17_mlp_gradient_by_finite_differences():
    p = CV.init_params(seed=4)
    rng = np.random.default_rng(9)
    X = rng.standard_normal((7, CV.NFEAT))
    T = rng.standard_normal((7, CV.NOUT))
    _, g = CV.loss_and_grad(p, X, T)
    flat, gflat = CV.flatten(p), CV.flatten(g)
    idx = rng.choice(flat.size, 60, replace=False)
    h = 1e-6
    for i in idx:
        a, b = flat.copy(), flat.copy()
        a[i] += h
        b[i] -= h
        fd = (CV.loss_and_grad(CV.unflatten(a), X, T)[0] - CV.loss_and_grad(CV.unflatten(b), X, T)[0]) / (2 * h)
        assert abs(fd - gflat[i]) < 1e-7 * max(1.0, abs(fd)), i


def test_adam_minimises_a_quadratic():
    """Adam on 1/2 ||y - t||^2 with a linear network drives the loss to ~0."""
    rng = np.random.default_rng(1)
    p = CV.init_params(seed=2)
    X = rng.standard_normal((64, CV.NFEAT))
    T = np.tanh(X[:, :2]) * 0.5
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    l0 = CV.loss_and_grad(p, X, T)[0]
    for t in range(1, 600):
        loss, g = CV.loss_and_grad(p, X, T)
        CV.adam_step(p, g, m, v, t, 3e-3)
    assert loss < 1e-3 * l0


def test_splitmix64_reference_output():
    """First output of SplitMix64 from state 0 (the published generator)."""
    assert CV.splitmix64(0) == 0xE220A8397B1DCDAF


def test_subset_is_a_uniform_choice():
    W, k = 32, 4
    counts = np.zeros(W)
    for call in range(4000):
        S = CV.subset(7, call, W, k)
        assert len(S) == k and len(set(S)) == k
        counts[S] += 1
    freq = counts / 4000
    assert np.all(np.abs(freq - k / W) < 0.03)


def test_features_at_the_trial():
    h1, chol, ecore, trial = gi.make_system(gi.SMALL.system)
    ham = O.build(h1, chol, ecore, trial, 4, 4, 0.005)
    f = CV.features(ham, trial.astype(complex), O)
    assert abs(f[4]) < 1e-24 and abs(f[5]) < 1e-24          # vbias = l at the trial
    assert abs(f[0] - 0.5 * np.sum(ham.lmf ** 2)) < 1e-12 and abs(f[1]) < 1e-14
    assert abs(f[6] - 1.0) < 1e-15 and abs(f[7]) < 1e-15     # <Psi|Psi> = 1
    ek = CV.exchange_energy(ham, trial.astype(complex), O)
    assert abs(ham.e_trial - (f[2] + f[0] + ek.real)) < 1e-12
    # at the trial sum_s Tr(K_s Psi_s) = sum_g sum_s Tr(T0 T0) = -2 EK
    assert abs(f[8] + 2.0 * ek.real) < 1e-12 * max(1.0, abs(ek)) and abs(f[9]) < 1e-14


@pytest.mark.parametrize("uhf", [False, True])
def test_first_order_exchange_feature_is_the_derivative_of_ek(uhf):
    """The tenth and ninth features carry the exchange energy to first order
    about the trial: along any walker path phi(e) through the trial, with Theta
    the Green's-function factor, d EK / de = -d Tr(K Theta) / de.  Central
    differences of the oracle's exchange energy (pinned to the 4-index ERI) and
    of the feature must agree; a wrong sign, a missing factor, the transposed
    K or the other spin's trial fail this."""
    m, na, nb = 6, 3, 2
    spec = gi.SystemSpec(m, na, nb, 9, tau=3.0, scale="literal", seed=5)
    h1, chol, _, trial = gi.make_system(spec)
    if uhf:
        q, _ = np.linalg.qr(np.random.default_rng(3).standard_normal((m, nb)))
        trial = np.hstack([trial[:, :na], q])
    ham = O.build(h1, chol, 0.2, trial, na, nb, 0.01)
    ks = CV.exchange_first_order_matrices(ham)
    rng = np.random.default_rng(11)
    d = rng.standard_normal((m, na + nb)) + 1j * rng.standard_normal((m, na + nb))
    eps = 1e-4
    plus, minus = trial + eps * d, trial - eps * d
    dek = CV.exchange_energy(ham, plus, O) - CV.exchange_energy(ham, minus, O)
    fp, fm = CV.features(ham, plus, O, ks), CV.features(ham, minus, O, ks)
    dlin = complex(fp[8] - fm[8], fp[9] - fm[9])
    assert abs(dek) > 1e-6
    assert abs(dek + dlin) < 1e-7 * abs(dek)


def test_adam_first_two_updates_in_closed_form():
    """Adam (Kingma & Ba 2015, Algorithm 1) from zero moments: with bias
    correction the first update is -lr g1 / (|g1| + eps) per component, and the
    second uses the corrected moments (b1 g1 + g2) / (1 + b1) and
    (b2 g1^2 + g2^2) / (1 + b2).  Gradients of very different scales (down to
    1e-9, where eps matters) separate eps outside the square root from eps
    inside it, and a missing bias correction moves the first step by ~3x."""
    rng = np.random.default_rng(5)
    p0 = CV.init_params(seed=6)
    scales = 10.0 ** rng.integers(-9, 2, size=CV.flatten(p0).size)
    g1 = CV.unflatten(rng.standard_normal(scales.size) * scales)
    g2 = CV.unflatten(rng.standard_normal(scales.size) * scales)
    lr, b1, b2, eps = 2e-3, 0.9, 0.999, 1e-8
    p = {k: v.copy() for k, v in p0.items()}
    m = {k: np.zeros_like(v) for k, v in p.items()}
    v = {k: np.zeros_like(x) for k, x in p.items()}
    CV.adam_step(p, g1, m, v, 1, lr)
    a, ga = CV.flatten(p0), CV.flatten(g1)
    step1 = a - lr * ga / (np.abs(ga) + eps)
    assert np.allclose(CV.flatten(p), step1, rtol=1e-14, atol=1e-16)
    CV.adam_step(p, g2, m, v, 2, lr)
    gb = CV.flatten(g2)
    mh = (b1 * ga + gb) / (1 + b1)
    vh = (b2 * ga ** 2 + gb ** 2) / (1 + b2)
    step2 = step1 - lr * mh / (np.sqrt(vh) + eps)
    assert np.allclose(CV.flatten(p), step2, rtol=1e-12, atol=1e-16)
