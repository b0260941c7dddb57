"""Pins of the oracle's free projection (the fp-AFQMC section) against Fock
space, Gauss-Hermite quadrature and closed forms.

A free-projection walker stands for c |phi>, carried as phi and the complex
log-amplitude a = log(c <Psi_T|phi>).  Every reference below is built from
Fock-space matrices (bit strings, explicit fermionic signs) and scipy's expm,
never from the oracle's own formulas, so a dropped term, a wrong sign of the
mean-field phase, a missing constant or an amplitude that moves under
re-orthogonalisation fails one of them.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from numpy.polynomial.hermite_e import hermegauss

from fockspace import FockSector, eri_from_chol
from oracle import afqmc_oracle as O
from test_oracle_pins import random_walker, tiny_system


def _state(sec, ct, phi, a, na):
    """c |phi> as a Fock vector, from the walker's orbitals and log-amplitude."""
    v = sec.slater(phi, na)
    return np.exp(a) / np.vdot(ct, v) * v


def _one_field_case(dt=0.05, seed=5):
    h1, chol, ecore, trial = tiny_system(m=4, na=2, nb=1, nchol=1, uhf=True, seed=seed)
    ham = O.build(h1, chol, ecore, trial, 2, 1, dt=dt)
    sec = FockSector(4, 2, 1)
    return ham, sec, h1, chol, ecore


def _exact_one_step(ham, sec, chol, vec):
    """exp(-dt (C - E_T)) F1 exp(dt/2 (v - m)^2) F1 vec in Fock space, F1 the
    half step of the shifted one-body operator: the Gaussian average of one
    free-projection step (exact for a single Cholesky vector)."""
    I = np.eye(sec.dim)
    F1 = scipy.linalg.expm(-0.5 * ham.dt * sec.one_body(ham.H1))
    V = sec.one_body(1j * chol[0]) - 1j * ham.lmf[0] * I
    hs = scipy.linalg.expm(0.5 * ham.dt * V @ V)
    return math.exp(-ham.dt * (ham.const - ham.e_trial)) * (F1 @ (hs @ (F1 @ vec)))


def _quadrature_walkers(ham, phi, a0, npts=60, order=24):
    nodes, wts = hermegauss(npts)
    wts = wts / math.sqrt(2 * math.pi)
    logo0 = O.overlap_theta(ham, phi)[0]
    out = []
    for x, wt in zip(nodes, wts):
        r = O.free_step_walker(ham, phi, logo0, a0, np.array([x]), taylor_order=order)
        assert r["flags"] == 0
        out.append((wt, r))
    return out


# FP1 -------------------------------------------------------------------------------
def test_fp1_one_step_gaussian_average_is_the_trotter_propagator():
    """sum_k omega_k c'_k |phi'_k> over Gauss-Hermite nodes equals the exact
    one-step operator (one Cholesky vector) applied to c |phi> in Fock space."""
    ham, sec, _, chol, _ = _one_field_case()
    ct = sec.slater(ham.trial, 2)
    phi = random_walker(4, 3, seed=7)
    a0 = complex(0.3, -1.1)
    acc = np.zeros(sec.dim, complex)
    for wt, r in _quadrature_walkers(ham, phi, a0):
        acc += wt * _state(sec, ct, r["phi"], r["log_amp"], 2)
    ref = _exact_one_step(ham, sec, chol, _state(sec, ct, phi, a0, 2))
    assert np.max(np.abs(acc - ref)) < 1e-11 * np.max(np.abs(ref))


# FP2 -------------------------------------------------------------------------------
def test_fp2_estimator_over_quadrature_walkers():
    """The estimator over the quadrature walkers (weights = quadrature weights)
    is the projected energy <Psi_T|H|Psi'>/<Psi_T|Psi'> of the exact one-step
    state, and its one-body part that of h + ecore."""
    ham, sec, h1, chol, ecore = _one_field_case(dt=0.08, seed=9)
    ct = sec.slater(ham.trial, 2)
    phi = random_walker(4, 3, seed=3)
    a0 = complex(-0.4, 2.0)
    qs = _quadrature_walkers(ham, phi, a0)
    wts = np.array([q[0] for q in qs])
    amps = np.array([q[1]["log_amp"] for q in qs])
    es = O.local_energies(ham, np.array([q[1]["phi"] for q in qs]))
    est = O.free_estimator(wts, amps, es, np.zeros(len(qs), np.uint32))
    psi = _exact_one_step(ham, sec, chol, _state(sec, ct, phi, a0, 2))
    H = sec.hamiltonian(h1, eri_from_chol(chol), ecore)
    H1 = sec.one_body(h1) + ecore * np.eye(sec.dim)
    den = np.vdot(ct, psi)
    assert abs(est["E"] - np.vdot(ct, H @ psi) / den) < 1e-10
    assert abs(est["N1"] / est["D"] - np.vdot(ct, H1 @ psi) / den) < 1e-10
    assert abs((est["N1"] + est["N2"]) / est["D"] - est["E"]) < 1e-12
    # D e^r is the Gaussian average of c' <Psi_T|phi'>: <Psi_T|Psi'>
    assert abs(est["D"] * math.exp(est["r"]) - den) < 1e-11 * abs(den)


# FP3 -------------------------------------------------------------------------------
def test_fp3_one_body_projection():
    """L = 0: free projection is the deterministic exp(-k dt h) evolution; the
    amplitude is <Psi_T|exp(-k dt (H - E_T))|phi0> and the energy the Fock
    projection, re-orthogonalising every 5 steps."""
    m, na, nb = 4, 2, 1
    h1, chol, ecore, trial = tiny_system(m=m, na=na, nb=nb, nchol=1, uhf=True)
    chol = np.zeros_like(chol)
    dt = 0.1
    ham = O.build(h1, chol, ecore, trial, na, nb, dt)
    sec = FockSector(m, na, nb)
    H = sec.one_body(h1) + ecore * np.eye(sec.dim)
    ct = sec.slater(ham.trial, na)
    phi0 = np.asarray(trial, complex) + random_walker(m, na + nb, seed=13, scale=0.3)
    c0 = sec.slater(phi0, na)
    phis = phi0[None].copy()
    logo = O.initial_logo(ham, phis)
    amps = O.initial_amplitudes(logo)
    for k in range(1, 31):
        phis, logo, amps, fl = O.free_propagate(ham, phis, logo, amps, np.zeros((1, 1)))
        assert fl[0] == 0
        if k % 5 == 0:
            phis, logo = O.reorthogonalize(ham, phis, logo)
        ck = scipy.linalg.expm(-k * dt * (H - ham.e_trial * np.eye(sec.dim))) @ c0
        ref = np.vdot(ct, ck)
        got = np.exp(amps[0])
        assert abs(got - ref) < 1e-11 * abs(ref)
        est = O.free_estimator(np.ones(1), amps, O.local_energies(ham, phis), fl)
        assert abs(est["E"] - np.vdot(ct, H @ ck) / ref) < 1e-10


# FP4 -------------------------------------------------------------------------------
def test_fp4_reorthogonalisation_keeps_the_walker_state():
    """Re-orthogonalisation rescales phi and log<Psi_T|phi> but the walker
    c |phi> (hence a) is unchanged."""
    ham, sec, _, _, _ = _one_field_case()
    ct = sec.slater(ham.trial, 2)
    phis = np.stack([random_walker(4, 3, seed=s, scale=0.9) for s in (1, 2)])
    logo = O.initial_logo(ham, phis)
    amps = np.array([0.2 + 0.7j, -1.0 - 2.5j])
    q, logo_q = O.reorthogonalize(ham, phis, logo)
    for w in range(2):
        before = _state(sec, ct, phis[w], amps[w], 2)
        after = _state(sec, ct, q[w], amps[w], 2)
        assert np.max(np.abs(before - after)) < 1e-12 * np.max(np.abs(before))
        assert abs(np.exp(logo_q[w]) - np.vdot(ct, sec.slater(q[w], 2))) < 1e-12 * abs(np.exp(logo_q[w]))


# FP5 -------------------------------------------------------------------------------
def test_fp5_estimator_definition():
    rng = np.random.default_rng(2)
    W = 7
    e = rng.standard_normal((W, 3)) + 1j * rng.standard_normal((W, 3))
    a = rng.standard_normal(W) * 3 + 1j * rng.uniform(-np.pi, np.pi, W)
    w = rng.uniform(0.5, 2.0, W)
    fl = np.zeros(W, np.uint32)
    est = O.free_estimator(w, a, e, fl)
    z = w * np.exp(a)
    assert abs(est["E"] - np.sum(z * e[:, 0]) / np.sum(z)) < 1e-12
    assert est["r"] == np.max(a.real) and est["n"] == W
    # a common shift of every amplitude leaves E unchanged and moves r
    est2 = O.free_estimator(w, a + (5.0 + 0.4j), e, fl)
    assert abs(est2["E"] - est["E"]) < 1e-12 and abs(est2["r"] - est["r"] - 5.0) < 1e-12
    # one walker: E is its local energy
    one = O.free_estimator(np.ones(1), a[:1], e[:1], fl[:1])
    assert abs(one["E"] - e[0, 0]) < 1e-12
    # flagged or zero-weight walkers do not count
    fl2 = fl.copy()
    fl2[1] = O.W_SINGULAR
    fl2[2] = O.W_NONFINITE
    w2 = w.copy()
    w2[3] = 0.0
    est3 = O.free_estimator(w2, a, e, fl2)
    keep = [0, 4, 5, 6]
    ref = O.free_estimator(w[keep], a[keep], e[keep], fl[keep])
    assert est3["n"] == 4 and abs(est3["E"] - ref["E"]) < 1e-13
    assert O.free_estimator(np.zeros(W), a, e, fl)["n"] == 0


# FP6 -------------------------------------------------------------------------------
def test_fp6_no_force_bias_and_no_phaseless_projection():
    """A free step applies the bare Gaussian field x (not x - xbar) and keeps
    walkers whose overlap ratio has a negative real part: its state is the
    determinant of B(x) phi from Fock-space exponentials, times the scalar
    exp(i sqrt(dt) x.l - dt (C - E_T))."""
    h1, chol, ecore, trial = tiny_system(m=4, na=2, nb=2, nchol=3, seed=8)
    ham = O.build(h1, chol, ecore, trial, 2, 2, dt=0.2)
    sec = FockSector(4, 2, 2)
    ct = sec.slater(ham.trial, 2)
    rng = np.random.default_rng(5)
    phi = random_walker(4, 4, seed=4, scale=0.8)
    logo = O.overlap_theta(ham, phi)[0]
    F1 = scipy.linalg.expm(-0.5 * ham.dt * sec.one_body(ham.H1))
    negative = 0
    for _ in range(12):
        x = 1.5 * rng.standard_normal(ham.nchol)
        r = O.free_step_walker(ham, phi, logo, logo, x, taylor_order=40)
        gen = sum(x[g] * sec.one_body(1j * chol[g]) for g in range(ham.nchol))
        scal = np.exp(1j * math.sqrt(ham.dt) * np.dot(x, ham.lmf) - ham.dt * (ham.const - ham.e_trial))
        ref = scal * (F1 @ (scipy.linalg.expm(-math.sqrt(ham.dt) * gen) @ (F1 @ sec.slater(phi, 2))))
        got = _state(sec, ct, r["phi"], r["log_amp"], 2)
        assert np.max(np.abs(got - ref)) < 1e-10 * np.max(np.abs(ref))
        s_ratio = np.exp(r["log_amp"] - logo)
        negative += s_ratio.real < 0
    assert negative > 0       # walkers the phaseless projection would have killed


def test_fp_nonfinite_field_is_flagged():
    ham, _, _, _, _ = _one_field_case()
    phi = random_walker(4, 3, seed=7)
    logo = O.overlap_theta(ham, phi)[0]
    r = O.free_step_walker(ham, phi, logo, logo, np.array([np.nan]))
    assert r["flags"] & O.W_NONFINITE
    r0 = O.free_step_walker(ham, phi, logo, logo, np.array([0.0]))
    assert np.array_equal(r["phi"], r0["phi"]) and r["log_amp"] == r0["log_amp"]
