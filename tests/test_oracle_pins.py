"""Pins of the CPU oracle against brute force, closed forms and identities.

None of these retypes the oracle's formulas: every reference value comes from
an independent route (Fock-space matrices built from bit strings, explicit
determinants, the 4-index ERI, Gauss-Hermite quadrature, finite differences,
scipy's expm), so a dropped term, a wrong sign, a transposed operand or a wrong
index in the oracle fails at least one of them.  The paper prints no worked
example for this path, so no pin is a printed number.
"""
import math

import numpy as np
import pytest
import scipy.linalg
from numpy.polynomial.hermite_e import hermegauss

import afqmc_inputs as gi
from fockspace import FockSector, eri_from_chol
from oracle import afqmc_oracle as O


def tiny_system(m=4, na=2, nb=2, nchol=5, scale="literal", seed=5, uhf=False, ecore=0.37):
    spec = gi.SystemSpec(m, na, nb, nchol, tau=3.0, scale=scale, seed=seed)
    h1, chol, _, trial = gi.make_system(spec)
    if uhf:
        rng = np.random.default_rng(seed + 11)
        qb, _ = np.linalg.qr(rng.standard_normal((m, nb)))
        trial = np.hstack([trial[:, :na], qb])
    return h1, chol, ecore, trial


def random_walker(m, ntot, seed=3, scale=0.4):
    rng = np.random.default_rng(seed)
    return (rng.standard_normal((m, ntot)) + 1j * rng.standard_normal((m, ntot))) * scale


CASES = [dict(m=4, na=2, nb=2), dict(m=4, na=2, nb=1, uhf=True), dict(m=5, na=2, nb=2, uhf=True)]


@pytest.fixture(scope="module", params=range(len(CASES)), ids=["M4-2a2b", "M4-2a1b-uhf", "M5-2a2b-uhf"])
def fock_case(request):
    c = CASES[request.param]
    h1, chol, ecore, trial = tiny_system(**c)
    na, nb = c["na"], c["nb"]
    ham = O.build(h1, chol, ecore, trial, na, nb, dt=0.01)
    sec = FockSector(c["m"], na, nb)
    H = sec.hamiltonian(h1, eri_from_chol(chol), ecore)
    return ham, sec, H


# P2 --------------------------------------------------------------------------------
def test_p2_hartree_fock_energy(fock_case):
    ham, sec, H = fock_case
    ct = sec.slater(ham.trial, ham.nalpha)
    e_fock = ct @ H @ ct / (ct @ ct)
    assert abs(ham.e_trial - e_fock) < 1e-11 * max(1, abs(e_fock))
    # closed form in terms of the trial's density matrices
    Ps = [ham.trial[:, sl] @ ham.trial[:, sl].T for sl in ham.spins()]
    L = ham.chol
    e = ham.ecore + sum(np.sum(ham.h1 * P) for P in Ps)
    coul = sum(np.einsum("gpq,pq->g", L, P) for P in Ps)
    e += 0.5 * np.sum(coul ** 2)
    e -= 0.5 * sum(np.einsum("gpq,qr,grs,sp->", L, P, L, P) for P in Ps)
    assert abs(ham.e_trial - e) < 1e-11 * max(1, abs(e))


# P3 --------------------------------------------------------------------------------
def test_p3_overlap_matches_determinants(fock_case):
    ham, sec, _ = fock_case
    phi = random_walker(ham.nbasis, ham.nalpha + ham.nbeta)
    logo, thetas, sing = O.overlap_theta(ham, phi)
    assert not sing
    ct = sec.slater(ham.trial, ham.nalpha)
    cp = sec.slater(phi, ham.nalpha)
    ov = np.vdot(ct, cp)
    assert abs(np.exp(logo) - ov) < 1e-12 * abs(ov)
    dets = np.prod([np.linalg.det(ham.trial[:, sl].T @ phi[:, sl]) for sl in ham.spins()])
    assert abs(np.exp(logo) - dets) < 1e-12 * abs(dets)


# P4 --------------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [3, 4])
def test_p4_local_energy_matches_fock_space(fock_case, seed):
    ham, sec, H = fock_case
    phi = random_walker(ham.nbasis, ham.nalpha + ham.nbeta, seed=seed)
    e, e1, e2 = O.local_energy(ham, phi)
    ct = sec.slater(ham.trial, ham.nalpha)
    cp = sec.slater(phi, ham.nalpha)
    ref = np.vdot(ct, H @ cp) / np.vdot(ct, cp)
    assert abs(e - ref) < 1e-10 * max(1, abs(ref))
    # the one-body part alone: H built from h and ecore only
    H1f = sec.one_body(ham.h1) + ham.ecore * np.eye(sec.dim)
    ref1 = np.vdot(ct, H1f @ cp) / np.vdot(ct, cp)
    assert abs(e1 - ref1) < 1e-10 * max(1, abs(ref1))


# P1 --------------------------------------------------------------------------------
def test_p1_cholesky_energy_equals_eri_energy():
    h1, chol, ecore, trial = tiny_system(m=6, na=3, nb=2, nchol=9, uhf=True)
    ham = O.build(h1, chol, ecore, trial, 3, 2, dt=0.01)
    phi = random_walker(6, 5, seed=9)
    _, e1, e2 = O.local_energy(ham, phi)
    _, thetas, _ = O.overlap_theta(ham, phi)
    eri = eri_from_chol(chol)  # eri[p,s,q,r] = (ps|qr)
    Gs = []
    for sl, th in zip(ham.spins(), thetas):
        psi = ham.trial[:, sl]
        Gs.append(psi @ th.T)  # G_pq = sum_i psi_pi theta_qi = <a+_p a_q>
    Gt = sum(Gs)
    coul = 0.5 * np.einsum("psqr,ps,qr->", eri, Gt, Gt)
    exch = -0.5 * sum(np.einsum("psqr,pr,qs->", eri, G, G) for G in Gs)
    assert abs(e2 - (coul + exch)) < 1e-11 * max(1, abs(e2))


# P7a -------------------------------------------------------------------------------
def test_p7a_mean_field_rewriting_in_fock_space(fock_case):
    """H = H1 + C - 1/2 sum_g (v_g - m_g)^2 with v_g = i sum L^g a+a, m_g = i l_g."""
    ham, sec, H = fock_case
    I = np.eye(sec.dim)
    rhs = sec.one_body(ham.H1).astype(complex) + ham.const * I
    for g in range(ham.nchol):
        V = sec.one_body(1j * ham.chol[g])
        D = V - 1j * ham.lmf[g] * I
        rhs -= 0.5 * D @ D
    assert np.max(np.abs(rhs - H)) < 1e-11


# P6 --------------------------------------------------------------------------------
def test_p6_thouless_for_the_two_body_generator(fock_case):
    """exp(-sqrt(dt) y.v) in Fock space equals the determinant of expm(A) phi,
    A = the oracle's orbital generator."""
    ham, sec, _ = fock_case
    rng = np.random.default_rng(21)
    y = rng.standard_normal(ham.nchol) + 0.3j * rng.standard_normal(ham.nchol)
    A = O.two_body_generator(ham, y)
    phi = random_walker(ham.nbasis, ham.nalpha + ham.nbeta, seed=5)
    gen = sum(y[g] * sec.one_body(1j * ham.chol[g]) for g in range(ham.nchol))
    lhs = scipy.linalg.expm(-math.sqrt(ham.dt) * gen) @ sec.slater(phi, ham.nalpha)
    rhs = sec.slater(scipy.linalg.expm(A) @ phi, ham.nalpha)
    assert np.max(np.abs(lhs - rhs)) < 1e-12 * np.max(np.abs(rhs))


# P7b -------------------------------------------------------------------------------
def test_p7b_hubbard_stratonovich_quadrature():
    """One Cholesky vector: the Gaussian average of the oracle's shifted
    propagator exp(i sqrt(dt) x l) det(expm(A(x)) phi) equals
    exp(dt/2 (v - m)^2) |phi> in Fock space."""
    h1, chol, ecore, trial = tiny_system(m=4, na=2, nb=1, nchol=1, uhf=True)
    ham = O.build(h1, chol, ecore, trial, 2, 1, dt=0.05)
    sec = FockSector(4, 2, 1)
    phi = random_walker(4, 3, seed=7)
    nodes, wts = hermegauss(60)
    wts = wts / math.sqrt(2 * math.pi)
    acc = np.zeros(sec.dim, complex)
    for x, wt in zip(nodes, wts):
        A = O.two_body_generator(ham, np.array([x + 0j]))
        scal = np.exp(1j * math.sqrt(ham.dt) * x * ham.lmf[0])
        acc += wt * scal * sec.slater(scipy.linalg.expm(A) @ phi, 2)
    V = sec.one_body(1j * chol[0]) - 1j * ham.lmf[0] * np.eye(sec.dim)
    ref = scipy.linalg.expm(0.5 * ham.dt * V @ V) @ sec.slater(phi, 2)
    assert np.max(np.abs(acc - ref)) < 1e-11 * np.max(np.abs(ref))


# P5 --------------------------------------------------------------------------------
def test_p5_force_bias_cancels_linear_term():
    """xbar = -grad_y ln S(y) at y = 0, S built from exact exponentials and
    determinants (no Green's function)."""
    h1, chol, ecore, trial = tiny_system(m=6, na=3, nb=2, nchol=4, uhf=True)
    ham = O.build(h1, chol, ecore, trial, 3, 2, dt=0.02)
    phi = np.asarray(trial, complex) + random_walker(6, 5, seed=2, scale=0.2)
    r = O.step_walker(ham, phi, 1.0, np.zeros(ham.nchol), fb_cap=0.0)
    xbar = r["xbar"]

    def lnS(y):
        A = O.two_body_generator(ham, y)
        val = 1j * math.sqrt(ham.dt) * np.sum(y * ham.lmf)
        for sl in ham.spins():
            psi = ham.trial[:, sl]
            val += np.log(np.linalg.det(psi.T @ scipy.linalg.expm(A) @ phi[:, sl]) /
                          np.linalg.det(psi.T @ phi[:, sl]))
        return val

    h = 1e-4
    grad = np.empty(ham.nchol, complex)
    for g in range(ham.nchol):
        e = np.zeros(ham.nchol, complex)
        e[g] = h
        grad[g] = (lnS(e) - lnS(-e)) / (2 * h)
    assert np.max(np.abs(-grad - xbar)) < 1e-8 * max(1.0, np.max(np.abs(xbar)))
    assert np.max(np.abs(xbar)) > 1e-3  # not a trivial zero


# P8 --------------------------------------------------------------------------------
def test_p8_importance_function_is_a_contour_shift():
    """int p(x) I(x) dx = int p(y) S(y) dy for one field (Gauss-Hermite)."""
    h1, chol, ecore, trial = tiny_system(m=4, na=2, nb=2, nchol=1)
    ham = O.build(h1, chol, ecore, trial, 2, 2, dt=0.05)
    phi = np.asarray(trial, complex) + random_walker(4, 4, seed=12, scale=0.3)
    logo0, _, _ = O.overlap_theta(ham, phi)
    nodes, wts = hermegauss(80)
    wts = wts / math.sqrt(2 * math.pi)
    lhs = sum(wt * O.step_walker(ham, phi, 1.0, np.array([x]), fb_cap=0.0)["I"]
              for x, wt in zip(nodes, wts))
    rhs = sum(wt * np.exp(O.overlap_ratio(ham, phi, logo0, np.array([x + 0j]))[2])
              for x, wt in zip(nodes, wts))
    r0 = O.step_walker(ham, phi, 1.0, np.array([0.0]), fb_cap=0.0)
    assert abs(r0["xbar"][0]) > 1e-3
    assert abs(lhs - rhs) < 1e-11 * abs(rhs)


# P9 / P10 / P11 / P12 ---------------------------------------------------------------
@pytest.fixture(scope="module")
def small_ham():
    spec = gi.SMALL
    h1, chol, ecore, trial = gi.make_system(spec.system)
    return O.build(h1, chol, ecore, trial, 4, 4, spec.dt)


def test_p9_reorthogonalisation_invariance(small_ham):
    ham = small_ham
    phis0 = gi.initial_walkers(ham.trial, 4, noise=0.05, seed=4)
    ra = O.run(ham, phis0.copy(), gi.FieldStream(0, 4, ham.nchol), 6, reortho_every=1)
    rb = O.run(ham, phis0.copy(), gi.FieldStream(0, 4, ham.nchol), 6, reortho_every=0)
    for a, b in zip(ra[3], rb[3]):
        assert np.allclose(a["weights"], b["weights"], rtol=1e-12, atol=0)
        assert np.allclose(a["energies"], b["energies"], rtol=1e-12, atol=0)
    # after MGS every spin block is orthonormal
    q = ra[0][0][:, :4]
    assert np.allclose(q.conj().T @ q, np.eye(4), atol=1e-13)


def test_p10_gauge_invariance(small_ham):
    ham = small_ham
    rng = np.random.default_rng(8)
    phi = gi.initial_walkers(ham.trial, 1, noise=0.1, seed=6)[0]
    C = [np.eye(4) + 0.3 * (rng.standard_normal((4, 4)) + 1j * rng.standard_normal((4, 4)))
         for _ in range(2)]
    phic = phi.copy()
    phic[:, :4] = phi[:, :4] @ C[0]
    phic[:, 4:] = phi[:, 4:] @ C[1]
    assert np.allclose(O.local_energy(ham, phi), O.local_energy(ham, phic), rtol=1e-11)
    x = np.random.default_rng(1).standard_normal(ham.nchol)
    ra = O.step_walker(ham, phi, 1.0, x)
    rb = O.step_walker(ham, phic, 1.0, x)
    assert abs(ra["weight"] - rb["weight"]) < 1e-12
    assert abs(ra["theta"] - rb["theta"]) < 1e-12


def test_p11_restricted_trial_keeps_spin_blocks_equal(small_ham):
    ham = small_ham
    phis, w, logo, recs = O.run(ham, gi.initial_walkers(ham.trial, 3),
                                gi.FieldStream(0, 3, ham.nchol), 6)
    assert np.max(np.abs(phis[:, :, :4] - phis[:, :, 4:])) < 1e-14


def test_p12_no_force_bias_at_the_trial(small_ham):
    ham = small_ham
    r = O.step_walker(ham, ham.trial.astype(complex), 1.0, np.zeros(ham.nchol), fb_cap=0.0)
    assert np.max(np.abs(r["xbar"])) < 1e-14
    # with x = 0 and walker = trial, theta is the phase of <Psi|B|Psi>: zero
    assert abs(r["theta"]) < 1e-14


# P13 -------------------------------------------------------------------------------
def test_p13_one_body_imaginary_time_evolution():
    """L = 0: walkers evolve by exp(-k dt h); the mixed energy follows the
    Fock-space projection and converges to the sum of the lowest orbital
    energies; the weight is the overlap growth times exp(-k dt (C - E_T))."""
    m, na, nb = 4, 2, 1
    h1, chol, ecore, trial = tiny_system(m=m, na=na, nb=nb, nchol=1, uhf=True)
    chol = np.zeros_like(chol)
    # trial: a small rotation of h's own lowest orbitals, so that the overlap
    # with exp(-k dt h) phi0 never crosses zero
    eps, vec = np.linalg.eigh(h1)
    rot = scipy.linalg.expm(0.2 * (np.triu(np.ones((m, m)), 1) - np.tril(np.ones((m, m)), -1)))
    trial = np.hstack([(vec @ rot)[:, :na], (vec @ rot.T)[:, :nb]])
    dt = 0.2
    ham = O.build(h1, chol, ecore, trial, na, nb, dt)
    sec = FockSector(m, na, nb)
    H = sec.one_body(h1) + ecore * np.eye(sec.dim)
    # a real starting walker keeps every overlap ratio real and positive (theta = 0)
    phi0 = np.asarray(trial, complex) + random_walker(m, na + nb, seed=13, scale=0.3).real
    ct = sec.slater(trial, na)
    c0 = sec.slater(phi0, na)
    phis = phi0[None].copy()
    w = np.ones(1)
    logo = O.initial_logo(ham, phis)
    for k in range(1, 41):
        phis, w, logo, _ = O.propagate(ham, phis, w, logo, np.zeros((1, 1)))
        ck = scipy.linalg.expm(-k * dt * H) @ c0
        e_ref = np.vdot(ct, H @ ck) / np.vdot(ct, ck)
        e = O.local_energy(ham, phis[0])[0]
        assert abs(e - e_ref) < 1e-10 * abs(e_ref)
        ratio = abs(np.vdot(ct, ck) / np.vdot(ct, c0) * np.exp(k * dt * ecore))
        w_ref = ratio * math.exp(-k * dt * (ham.const - ham.e_trial))
        assert abs(w[0] - w_ref) < 1e-10 * w_ref
    for k in range(400):  # long run: columns need re-orthogonalising
        phis, w, logo, _ = O.propagate(ham, phis, w, logo, np.zeros((1, 1)))
        phis, logo = O.reorthogonalize(ham, phis, logo)
    e = O.local_energy(ham, phis[0])[0]
    eps = np.linalg.eigvalsh(h1)
    assert abs(e.real - (ecore + eps[:na].sum() + eps[:nb].sum())) < 1e-6


# P14 -------------------------------------------------------------------------------
def test_p14_taylor_error_bound():
    rng = np.random.default_rng(4)
    for norm in (0.05, 0.3, 1.0):
        A = rng.standard_normal((12, 12)) + 1j * rng.standard_normal((12, 12))
        A = 0.5 * (A + A.T)
        A *= norm / np.linalg.norm(A, 2)
        phi = rng.standard_normal((12, 3)) + 0j
        err = np.linalg.norm(O.taylor_apply(A, phi, 6) - scipy.linalg.expm(A) @ phi, 2)
        bound = norm ** 7 / math.factorial(7) * math.exp(norm) * np.linalg.norm(phi, 2)
        assert err <= bound * (1 + 1e-6) + 1e-15
        assert err > 0.01 * bound  # the truncation is real, not absent


def test_mgs_factorisation():
    rng = np.random.default_rng(2)
    a = rng.standard_normal((9, 4)) + 1j * rng.standard_normal((9, 4))
    q, r = O.mgs(a)
    assert np.allclose(q @ r, a, atol=1e-13)
    assert np.allclose(q.conj().T @ q, np.eye(4), atol=1e-13)
    assert np.all(np.diag(r).real > 0) and np.allclose(np.tril(r, -1), 0)
    # same factors as a Householder QR with the sign fixed
    qh, rh = np.linalg.qr(a)
    ph = np.diag(rh) / np.abs(np.diag(rh))
    assert np.allclose(q, qh * ph, atol=1e-12)


def test_estimator_definition():
    w = np.array([1.0, 0.0, 2.0])
    e = np.array([[1 + 1j, 0.5, 0.5 + 1j], [9, 9, 9], [3 - 1j, 1, 2 - 1j]], complex)
    est = O.estimator(w, e)
    assert est["ENumer"] == pytest.approx(7.0)
    assert est["EDenom"] == pytest.approx(3.0)
    assert est["E1Body"] == pytest.approx(2.5)
    assert est["E2Body"] == pytest.approx(4.5)


def test_singular_walker_gets_zero_weight(small_ham):
    ham = small_ham
    # an alpha orbital with exactly zero overlap with the trial: <Psi_T|phi> = 0
    phi = ham.trial.astype(complex).copy()
    phi[:, 0] = 0.0
    r = O.step_walker(ham, phi, 1.0, np.zeros(ham.nchol))
    assert r["weight"] == 0.0 and r["flags"] & O.W_SINGULAR


def test_generator_recipe():
    h1, chol, ecore, trial = gi.make_system(gi.SMALL.system)
    assert np.allclose(h1, h1.T) and np.all(np.diff(np.diag(h1)) >= 0)
    assert np.allclose(chol, chol.transpose(0, 2, 1))
    ratio = np.linalg.norm(chol[40]) / np.linalg.norm(chol[20])
    assert 0.2 < ratio < 0.6  # exp(-20/20) ~ 0.37 up to sampling noise
    assert np.allclose(trial[:, :4].T @ trial[:, :4], np.eye(4), atol=1e-12)
    assert gi.batching_walker_counts() == [428, 102, 144, 170, 145, 423, 454, 325,
                                           81, 106, 213, 258, 342, 279, 182, 135]


def test_counter_recipe_generator():
    """The counter recipe's Cholesky vectors: symmetric, standardised bracket of
    mean 0 and variance 1, scaled by exp(-g/tau) * scale, the same entries
    whatever subset of vectors is drawn, and SplitMix64's published first output."""
    import math
    m, g, tau, scale = 30, 40, 12.0, 1.0 / 30
    L = gi.make_chol_counter(11, m, g, tau, scale)
    assert np.array_equal(L, L.transpose(0, 2, 1))
    z = np.concatenate([L[k][np.triu_indices(m)] / (math.exp(-k / tau) * scale) for k in range(g)])
    assert abs(z.mean()) < 0.02 and abs(z.std() - 1.0) < 0.02 and np.abs(z).max() <= 2 * math.sqrt(3) + 1e-12
    sub = gi.make_chol_counter(11, m, g, tau, scale, gammas=[3, 17])
    assert np.array_equal(sub[0], L[3]) and np.array_equal(sub[1], L[17])
    assert int(gi.splitmix64_outputs(0, np.array([0], dtype=np.uint64))[0]) == 0xE220A8397B1DCDAF
    spec = gi.SystemSpec(m, 3, 3, g, tau=tau, seed=11, recipe="counter")
    h1, chol, ecore, trial = gi.make_system(spec)
    assert np.array_equal(chol, L)
    h1b, ecb, trb = gi.make_system_without_chol(spec)
    assert np.array_equal(h1, h1b) and np.array_equal(trial, trb)


def test_comb_population_control():
    """The comb keeps W walkers and the total weight; each walker gets floor or
    ceil of W w_i / Wt copies, zero-weight walkers none, and averaged over the
    offset u the copies are exactly W w_i / Wt."""
    rng = np.random.default_rng(8)
    W = 37
    w = rng.exponential(1.0, W)
    w[[3, 11]] = 0.0
    total = np.cumsum(w)[-1]
    mean = np.zeros(W)
    grid = (np.arange(4000) + 0.5) / 4000
    for u in grid:
        parents, nw = O.comb(w, u)
        n = np.bincount(parents, minlength=W)
        assert n.sum() == W and np.allclose(nw, total / W)
        assert np.all(n >= np.floor(W * w / total) - 1e-12) and np.all(n <= np.ceil(W * w / total) + 1e-12)
        assert n[3] == 0 and n[11] == 0
        assert np.all(np.diff(parents) >= 0)
        mean += n / len(grid)
    assert np.max(np.abs(mean - W * w / total)) < 2e-3


# P18 / P19: the phaseless projection and the force-bias cap ---------------------------
class FockReference:
    """Everything the weight update needs, built in Fock space only: the
    Hamiltonian from the 4-index ERI, the mean-field shift and E_T as trial
    expectations, the one-body operator of the shifted split as
    H - C + 1/2 sum_g (v_g - m_g)^2, the force bias as the mixed expectation of
    the bare two-body generator, and the overlap ratio S of eq. ovlp_ratio from
    dense exponentials (no Green's function, no Thouless, no Taylor series)."""

    def __init__(self, h1, chol, ecore, trial, na, nb, dt):
        m = h1.shape[0]
        self.sec = sec = FockSector(m, na, nb)
        self.dt = dt
        self.G = chol.shape[0]
        H = sec.hamiltonian(h1, eri_from_chol(chol), ecore)
        self.ct = sec.slater(trial, na)
        nrm = self.ct @ self.ct
        self.V = [sec.one_body(1j * chol[g]) for g in range(self.G)]
        self.l = np.array([(self.ct @ sec.one_body(chol[g]) @ self.ct) / nrm for g in range(self.G)])
        self.e_trial = float((self.ct @ H @ self.ct) / nrm)
        self.C = ecore - 0.5 * float(np.sum(self.l ** 2))
        Id = np.eye(sec.dim)
        self.D = [self.V[g] - 1j * self.l[g] * Id for g in range(self.G)]
        H1 = H - self.C * Id + 0.5 * sum(d @ d for d in self.D)
        self.half = scipy.linalg.expm(-0.5 * dt * H1)

    def xbar(self, phi, na):
        cp = self.sec.slater(phi, na)
        den = np.vdot(self.ct, cp)
        return np.array([math.sqrt(self.dt) * np.vdot(self.ct, d @ cp) / den for d in self.D])

    def S(self, phi, na, y):
        cp = self.sec.slater(phi, na)
        two = scipy.linalg.expm(-math.sqrt(self.dt) * sum(y[g] * self.D[g] for g in range(self.G)))
        return np.vdot(self.ct, self.half @ two @ self.half @ cp) / np.vdot(self.ct, cp)


@pytest.fixture(scope="module")
def phase_case():
    """Strong coupling (literal scale, dt = 0.3), two Cholesky vectors, an open
    shell with different alpha and beta trials, a complex walker."""
    m, na, nb, g, seed = 4, 2, 1, 2, 5
    h1, chol, ecore, trial = tiny_system(m=m, na=na, nb=nb, nchol=g, seed=seed, uhf=True)
    dt = 0.3
    ham = O.build(h1, chol, ecore, trial, na, nb, dt)
    ref = FockReference(h1, chol, ecore, trial, na, nb, dt)
    rng = np.random.default_rng(seed)
    phi = trial.astype(complex) + 0.5 * (rng.standard_normal((m, na + nb)) + 1j * rng.standard_normal((m, na + nb)))
    return ham, ref, phi


def _fock_weight(ref, phi, na, x, xbar, w0):
    """w0 |I| max(0, cos arg S) exp(-dt (C - E_T)) with S and I from Fock space,
    I = S exp(x.xbar - xbar.xbar / 2) (bilinear, eq. of the importance function)."""
    S = ref.S(phi, na, x - xbar)
    I = S * np.exp(np.sum(x * xbar) - 0.5 * np.sum(xbar * xbar))
    return w0 * abs(I) * max(0.0, math.cos(np.angle(S))) * math.exp(-ref.dt * (ref.C - ref.e_trial)), S, I


def test_p18_phaseless_projection_uses_the_phase_of_S(phase_case):
    """theta = arg S (Sec. 2: the phaseless projection of the overlap ratio),
    not arg I: one field where cos(arg S) < 0 < cos(arg I) must kill the walker
    (weight exactly 0, W_DEAD), one where both are positive must give
    w |I| cos(arg S) exp(-dt (C - E_T)), and the S, I the oracle reports must be
    the Fock-space ones.  The Taylor order is raised so that the truncated
    series equals the exponential to rounding."""
    ham, ref, phi = phase_case
    na = ham.nalpha
    xb = ref.xbar(phi, na)
    assert np.max(np.abs(xb.real)) > 0.05 and np.max(np.abs(xb.imag)) > 0.05  # arg I != arg S
    rng = np.random.default_rng(17)
    killed = kept = None
    for _ in range(400):
        x = 2.0 * rng.standard_normal(ham.nchol)
        wref, S, I = _fock_weight(ref, phi, na, x, xb, 0.75)
        cs, ci = math.cos(np.angle(S)), math.cos(np.angle(I))
        if killed is None and cs < -0.2 and ci > 0.2:
            killed = (x, S, I)
        if kept is None and cs > 0.2 and ci > 0.2 and abs(cs - ci) > 0.3:
            kept = (x, S, I, wref)
        if killed is not None and kept is not None:
            break
    assert killed is not None and kept is not None
    x, S, I = killed
    r = O.step_walker(ham, phi, 0.75, x, fb_cap=0.0, taylor_order=40)
    assert np.max(np.abs(r["xbar"] - xb)) < 1e-12
    assert abs(r["S"] - S) < 1e-10 * abs(S) and abs(r["I"] - I) < 1e-10 * abs(I)
    assert r["weight"] == 0.0 and r["flags"] & O.W_DEAD
    x, S, I, wref = kept
    r = O.step_walker(ham, phi, 0.75, x, fb_cap=0.0, taylor_order=40)
    assert not r["flags"] & O.W_DEAD
    assert abs(r["theta"] - np.angle(S)) < 1e-10
    assert abs(r["weight"] - wref) < 1e-10 * wref


def test_p19_force_bias_cap_rescales_the_modulus(phase_case):
    """The cap (reading R4): a component whose modulus exceeds c is rescaled to
    modulus c with its phase unchanged, the others are untouched, and the capped
    force bias is the one that shifts the field and enters I."""
    ham, ref, phi = phase_case
    na = ham.nalpha
    xb = ref.xbar(phi, na)
    mags = np.abs(xb)
    c = 0.5 * (mags.min() + mags.max())
    assert mags.min() < c < mags.max()
    xc = np.where(mags > c, c * xb / mags, xb)
    x = np.array([0.3, -0.4])
    r = O.step_walker(ham, phi, 1.0, x, fb_cap=c, taylor_order=40)
    assert np.max(np.abs(r["xbar"] - xc)) < 1e-12
    big = mags > c
    assert np.allclose(np.abs(r["xbar"][big]), c, rtol=1e-13, atol=0)
    assert np.allclose(np.angle(r["xbar"][big]), np.angle(xb[big]), rtol=0, atol=1e-12)
    wref, S, I = _fock_weight(ref, phi, na, x, xc, 1.0)
    assert abs(r["S"] - S) < 1e-10 * abs(S) and abs(r["I"] - I) < 1e-10 * abs(I)
    assert abs(r["weight"] - wref) < 1e-10 * wref


# P20: blocks, comb and E_T feedback ------------------------------------------------
def test_p20_blocks_without_comb_or_feedback_repeat_the_step_loop(small_ham):
    ham = small_ham
    phis0 = gi.initial_walkers(ham.trial, 5, noise=0.05, seed=6)
    ra = O.run(ham, phis0.copy(), gi.FieldStream(2, 5, ham.nchol), 9, reortho_every=5)
    rb = O.run_blocks(ham, phis0.copy(), gi.FieldStream(2, 5, ham.nchol), 3, 3, offsets=None, feedback=False)
    flat = [e for blk in rb[3] for e in blk["est"]]
    assert len(flat) == 9
    for a, b in zip(ra[3], flat):
        assert a["est"] == b
    assert all(blk["e_shift"] == ham.e_trial for blk in rb[3])


def test_p20_feedback_scales_weights_only(small_ham):
    """E_T enters the weight update as the factor exp(dt E_T), common to every
    walker: with feedback the per-step mixed energies and the comb's choices are
    those of the run without it, and the total weight differs by exactly
    exp(dt sum_steps (E_T,step - E_HF)).  A wrong sign or a missing dt in the
    E_T factor fails the last check; the block energy it feeds back is the
    ratio of the block's summed records."""
    ham = small_ham
    W, nb, ns = 6, 4, 3
    phis0 = gi.initial_walkers(ham.trial, W, noise=0.05, seed=7)
    offs = np.random.default_rng(21).random(nb)
    # a shifted starting E_T makes the first feedback step large
    e0 = ham.e_trial + 0.7
    fa = O.run_blocks(ham, phis0.copy(), gi.FieldStream(3, W, ham.nchol), nb, ns, offs, feedback=False, e_shift=e0)
    fb = O.run_blocks(ham, phis0.copy(), gi.FieldStream(3, W, ham.nchol), nb, ns, offs, feedback=True, e_shift=e0)
    log_ratio = 0.0
    for ba, bb in zip(fa[3], fb[3]):
        assert np.array_equal(ba["parents"], bb["parents"])
        for ea, eb in zip(ba["est"], bb["est"]):
            assert eb["ENumer"] / eb["EDenom"] == pytest.approx(ea["ENumer"] / ea["EDenom"], rel=1e-12)
        log_ratio += ham.dt * ns * (bb["e_shift"] - e0)
    assert fb[3][0]["e_shift"] == e0
    for prev, nxt in zip(fb[3][:-1], fb[3][1:]):
        num = sum(e["ENumer"] for e in prev["est"])
        den = sum(e["EDenom"] for e in prev["est"])
        assert nxt["e_shift"] == pytest.approx(num / den, rel=1e-14)
        # the block estimate sits near the trial energy, far from the shifted start
        assert abs(nxt["e_shift"] - ham.e_trial) < 0.1
    assert np.sum(fb[1]) / np.sum(fa[1]) == pytest.approx(np.exp(log_ratio), rel=1e-11)
