"""CPU oracle for the phaseless-AFQMC walker step.

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.  The product path
(the HIP library and its Python binding) never calls it and shares no code with
it; the only common import is the seeded input generator, which holds none of
the method's arithmetic.

Plain numpy complex128 / float64, one walker at a time, library primitives only
(matmul, einsum, slogdet, solve, scipy expm).  It follows the paper's
"Theory of AFQMC" section (arXiv:2406.16238, Sec. 2):

* Hamiltonian, eq. (qcham), Cholesky factorisation, eq. (chol_decomp), and the
  rewriting H = v0 - 1/2 sum_g v_g^2 with v_g = i sum_pq L^g_pq a+_p a_q
  (the equations after eq. chol_decomp and eq. chol);
* symmetric Trotter split, eq. (trotter), and the HS propagator B(x), eq. (Bprop);
* walker expansion and mixed energy estimator, eq. (Eloc);
* propagation with the shifted field, eq. (propagate), the weight update,
  eq. (weight_update), the force bias, eq. (fb), the phaseless and hybrid
  importance functions and the overlap ratio S, eq. (ovlp_ratio), theta = arg S.

Where the paper defers to the literature (Green's function, half rotation,
local energy) the oracle uses the textbook identities: Wick's theorem for a
single determinant and Thouless' theorem for exponentials of one-body
operators.  Readings where the paper is silent or garbled:

R1  Force-bias sign.  With B = exp(-sqrt(dt) x.v) as printed, the bias that
    cancels the linear term of ln I is xbar = +sqrt(dt) (<v> - <v>_T)
    = i sqrt(dt) (vbias - l); the printed minus sign is taken as a typo.
R2  The mean-field shift m_g = <v_g>_T = i l_g enters through the exact
    rewriting H = H1 + C - 1/2 sum_g (v_g - m_g)^2 with
    H1 = v0 + sum_g l_g L^g and C = ecore - 1/2 sum_g l_g^2, and through the
    scalar exp(i sqrt(dt) y.l) of exp(-sqrt(dt) y.(v - m)) inside S.
R3  theta = arg S (not arg I).
R4  Force-bias cap: |xbar_g| > c  =>  xbar_g <- c xbar_g / |xbar_g|, c = 1 by
    default; c <= 0 disables it.
R5  The two-body exponential is a Taylor series of order 6.
R6  Energy shift E_T = E_HF (the trial's own local energy) unless the block
    loop (R13) moves it.
R7  No hybrid-energy capping; a walker with cos(theta) <= 0 gets weight
    exactly 0 and keeps propagating (until a comb, R11, drops it).
R8  The mixed estimator is normalised by sum_i w_i and uses Re E_loc.
R9  Re-orthogonalisation: modified Gram-Schmidt per spin block with positive
    real R_ii; log<Psi_T|phi> decreases by sum log R_ii.
R10 The overlap is carried as a complex logarithm; S is formed from the
    logarithms of the walker's overlap before and after the step, both
    recomputed from the determinants.
R11 Population control (named, not specified): a comb over the cumulative
    weights with one uniform offset; every new walker carries the mean weight.
R12 Free projection (the fp-AFQMC section): fields from the plain Gaussian,
    mean-field subtraction only.  A walker stands for c |phi> with c the scalar
    the shifted propagator accumulates; it carries the complex logarithm
    a = log(c <Psi_T|phi>).  A step adds log S - dt (C - E_T) to a (S as in
    eq. ovlp_ratio with y = x); re-orthogonalisation changes phi and
    log<Psi_T|phi> but not a.  E(tau) = sum_w w_w e^{a_w} E_loc,w /
    sum_w w_w e^{a_w} (complex), summed with the reference shift
    r = max Re a_w over the walkers that count (w_w > 0, no singular or
    non-finite flag); E_T = E_HF only keeps the amplitudes of order one.  No
    walker is killed, capped or resampled.
R13 Blocks (the simulation loop of Sec. 3.1 runs propagation, stabilisation,
    population control and estimators and writes its output once per block):
    a block is a fixed number of steps, each measuring the mixed estimator;
    after the last step of a block one comb (R11) resamples the walkers and
    E_T becomes the block's own estimate sum_k ENumer_k / sum_k EDenom_k (the
    paper does not say how E_T is fed back; a global E_T only scales every
    weight alike, so the estimator does not depend on it).
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.linalg

# per-walker status bits (same meaning as the library's flag word)
W_SINGULAR = 1
W_NONFINITE = 2
W_DEAD = 4


@dataclasses.dataclass
class OracleHamiltonian:
    """Hamiltonian, trial and everything derived from them at set-up."""

    h1: np.ndarray          # [M,M] one-body integrals
    chol: np.ndarray        # [G,M,M] Cholesky vectors L^g (real symmetric)
    ecore: float
    trial: np.ndarray       # [M, Na+Nb] real, alpha columns first
    nalpha: int
    nbeta: int
    dt: float
    # derived
    v0: np.ndarray = None          # h - 1/2 sum_g L^g L^g
    lmf: np.ndarray = None         # l_g = sum_s Tr(L^g P_s) (real); m_g = i l_g
    H1: np.ndarray = None          # v0 + sum_g l_g L^g
    const: float = 0.0             # ecore - 1/2 sum_g l_g^2
    B1: np.ndarray = None          # expm(-dt/2 H1)
    lhalf: list = None             # per spin [G, N_s, M]: Psi_s^T L^g
    hhalf: list = None             # per spin [N_s, M]: Psi_s^T h
    e_trial: float = 0.0           # E_T = E_HF

    @property
    def nbasis(self) -> int:
        return self.h1.shape[0]

    @property
    def nchol(self) -> int:
        return self.chol.shape[0]

    def spins(self):
        """Column slices of the alpha and beta blocks."""
        return (slice(0, self.nalpha), slice(self.nalpha, self.nalpha + self.nbeta))


def build(h1, chol, ecore, trial, nalpha, nbeta, dt) -> OracleHamiltonian:
    """Set-up quantities (theory section: v0 after the Cholesky rewrite, the
    mean-field shift of eq. fb, the Trotter one-body factor of eq. Bprop)."""
    ham = OracleHamiltonian(np.asarray(h1, float), np.asarray(chol, float), float(ecore),
                            np.asarray(trial, float), int(nalpha), int(nbeta), float(dt))
    L = ham.chol
    G, M = L.shape[0], L.shape[1]
    # sum_r (pr|rq) = sum_g sum_r L^g_pr L^g_rq = sum_g (L^g L^g)_pq, written as
    # one product over the combined index (g, r)
    exch = L.transpose(1, 0, 2).reshape(M, G * M) @ L.reshape(G * M, M)
    ham.v0 = ham.h1 - 0.5 * exch
    # mean-field shift: <v_g>_T = i sum_s sum_pq L^g_pq <a+_p a_q>_T, with the
    # trial's density matrix P_s = Psi_s Psi_s^T (orthonormal real orbitals)
    lmf = np.zeros(ham.nchol)
    ham.lhalf, ham.hhalf = [], []
    for sl in ham.spins():
        psi = ham.trial[:, sl]
        P = psi @ psi.T
        lmf += L.reshape(G, M * M) @ P.ravel()
        ham.lhalf.append(np.matmul(psi.T, L))            # [G, N_s, M]
        ham.hhalf.append(psi.T @ ham.h1)
    ham.lmf = lmf
    ham.H1 = ham.v0 + np.tensordot(lmf, L, axes=1)
    ham.const = ham.ecore - 0.5 * float(lmf @ lmf)
    ham.B1 = scipy.linalg.expm(-0.5 * ham.dt * ham.H1)
    e, _, _ = local_energy(ham, ham.trial.astype(np.complex128))
    ham.e_trial = float(e.real)
    return ham


# ---- overlap and Green's function ---------------------------------------------

def overlap_theta(ham: OracleHamiltonian, phi: np.ndarray):
    """log<Psi_T|phi> and Theta_s = phi_s (Psi_s^T phi_s)^-1 per spin.

    <Psi_T|phi> = prod_s det(Psi_s^T phi_s); the mixed Green's function is
    G^s_pq = <a+_p a_q> = sum_i Psi_pi Theta_qi.
    Returns (logO, [Theta_a, Theta_b], singular_flag)."""
    logo = 0.0 + 0.0j
    thetas = []
    singular = False
    for sl in ham.spins():
        psi = ham.trial[:, sl]
        ph = phi[:, sl]
        if ph.shape[1] == 0:
            thetas.append(np.zeros_like(ph))
            continue
        O = psi.T @ ph
        sign, logabs = np.linalg.slogdet(O)
        if sign == 0 or not np.isfinite(logabs):
            singular = True
            thetas.append(np.zeros_like(ph))
            continue
        logo += logabs + 1j * np.angle(sign)
        # Theta O = phi  <=>  O^T Theta^T = phi^T
        thetas.append(np.linalg.solve(O.T, ph.T).T)
    return logo, thetas, singular


def force_bias(ham: OracleHamiltonian, thetas) -> np.ndarray:
    """vbias_g = sum_s sum_pq L^g_pq G^s_pq = sum_s Tr(Ltilde^{g s} Theta_s);
    <v_g> = i vbias_g (eq. fb numerator before the mean-field subtraction)."""
    vb = np.zeros(ham.nchol, dtype=np.complex128)
    for s, th in enumerate(thetas):
        lh = ham.lhalf[s].reshape(ham.nchol, -1)      # [G, (i, q)]
        t = th.T.ravel()                              # Theta_qi ordered as (i, q)
        vb += lh @ np.ascontiguousarray(t.real) + 1j * (lh @ np.ascontiguousarray(t.imag))
    return vb


# ---- local energy ---------------------------------------------------------------

def local_energy(ham: OracleHamiltonian, phi: np.ndarray):
    """E_loc = <Psi_T|H|phi>/<Psi_T|phi> (eq. Eloc) for one walker.

    Wick's theorem for a single determinant with the Cholesky form of the ERI:
      E1 = ecore + sum_s Tr(htilde_s Theta_s)
      EJ = 1/2 sum_g vbias_g^2
      EK = -1/2 sum_g sum_s Tr(T^{gs} T^{gs}),  T^{gs} = Ltilde^{gs} Theta_s
    Returns (E, E1, E2) with E2 = EJ + EK, all complex."""
    _, thetas, singular = overlap_theta(ham, phi)
    if singular:
        return 0j, 0j, 0j
    e1 = ham.ecore + 0j
    for s, th in enumerate(thetas):
        e1 += np.einsum("iq,qi->", ham.hhalf[s], th)
    vb = force_bias(ham, thetas)
    ej = 0.5 * np.sum(vb * vb)
    ek = 0j
    for s, th in enumerate(thetas):
        lh = ham.lhalf[s]
        if lh.shape[1] == 0:
            continue
        G, n, M = lh.shape
        lh2 = lh.reshape(G * n, M)
        tr, ti = np.ascontiguousarray(th.real), np.ascontiguousarray(th.imag)
        T = (lh2 @ tr + 1j * (lh2 @ ti)).reshape(G, n, n)
        ek += -0.5 * np.einsum("gij,gji->", T, T)
    e2 = ej + ek
    return e1 + e2, e1, e2


def local_energies(ham: OracleHamiltonian, phis: np.ndarray) -> np.ndarray:
    """[W,3] complex: (E, E1, E2) per walker."""
    return np.array([local_energy(ham, p) for p in phis], dtype=np.complex128)


def estimator(weights: np.ndarray, energies: np.ndarray) -> dict:
    """ENumer, EDenom, E1Body, E2Body of the mixed estimator (the energy
    estimator record of the Estimators section).  Walkers with zero weight do
    not contribute."""
    live = weights > 0
    w = weights[live]
    e = energies[live]
    return {"ENumer": float(np.sum(w * e[:, 0].real)),
            "EDenom": float(np.sum(w)),
            "E1Body": float(np.sum(w * e[:, 1].real)),
            "E2Body": float(np.sum(w * e[:, 2].real))}


# ---- propagation -----------------------------------------------------------------

def taylor_apply(A: np.ndarray, phi: np.ndarray, order: int = 6) -> np.ndarray:
    """sum_{n=0}^{order} A^n phi / n!  (truncated series for exp(A) phi)."""
    term = phi.copy()
    acc = phi.copy()
    for n in range(1, order + 1):
        term = (A @ term) / n
        acc = acc + term
    return acc


def two_body_generator(ham: OracleHamiltonian, y: np.ndarray) -> np.ndarray:
    """A = -sqrt(dt) sum_g y_g (i L^g): the orbital matrix of
    exp(-sqrt(dt) y.v) by Thouless' theorem (sqrt(dt) times V_HS)."""
    L2 = ham.chol.reshape(ham.nchol, -1)
    vhs = -1j * ((np.ascontiguousarray(y.real) @ L2) + 1j * (np.ascontiguousarray(y.imag) @ L2))
    return np.sqrt(ham.dt) * vhs.reshape(ham.nbasis, ham.nbasis)


def overlap_ratio(ham: OracleHamiltonian, phi, logo0, y, taylor_order=6):
    """Apply B(y) = exp(-dt/2 H1) exp(-sqrt(dt) y.(v - m)) exp(-dt/2 H1) to phi
    (eq. Bprop with the mean-field shift) and return
    (phi', log<Psi_T|phi'>, log S, singular) with
    S = <Psi_T|B(y)|phi>/<Psi_T|phi> (eq. ovlp_ratio); the scalar
    exp(sqrt(dt) y.m) = exp(i sqrt(dt) y.l) is part of S."""
    A = two_body_generator(ham, y)
    phi1 = ham.B1 @ phi
    phi2 = taylor_apply(A, phi1, taylor_order)
    phi3 = ham.B1 @ phi2
    logo1, _, sing1 = overlap_theta(ham, phi3)
    log_s = (logo1 - logo0) + 1j * np.sqrt(ham.dt) * np.sum(y * ham.lmf)
    return phi3, logo1, log_s, sing1


def step_walker(ham: OracleHamiltonian, phi, weight, x, fb_cap=1.0, taylor_order=6, e_shift=None):
    """One phaseless step for one walker: eqs. (propagate), (weight_update),
    (fb), the hybrid importance function and (ovlp_ratio).  `e_shift` is E_T
    (None: the trial energy, reading R6).

    Returns a dict with the new phi, weight, logO and flags, and the
    intermediate quantities (xbar, S, I, theta) for the pins."""
    sqdt = np.sqrt(ham.dt)
    flags = 0
    logo0, thetas, singular = overlap_theta(ham, phi)
    if singular:
        return {"phi": phi.copy(), "weight": 0.0, "logo": logo0, "flags": W_SINGULAR,
                "xbar": np.zeros(ham.nchol, complex), "S": 0j, "I": 0j, "theta": 0.0}
    x = np.asarray(x, dtype=float)
    if not np.all(np.isfinite(x)):
        flags |= W_NONFINITE
        x = np.zeros_like(x)
    vb = force_bias(ham, thetas)
    xbar = 1j * sqdt * (vb - ham.lmf)
    if fb_cap > 0:
        mag = np.abs(xbar)
        big = mag > fb_cap
        xbar[big] = fb_cap * xbar[big] / mag[big]
    y = x - xbar
    phi3, logo1, log_s, sing1 = overlap_ratio(ham, phi, logo0, y, taylor_order)
    if sing1:
        return {"phi": phi3, "weight": 0.0, "logo": logo0, "flags": flags | W_SINGULAR,
                "xbar": xbar, "S": 0j, "I": 0j, "theta": 0.0}
    S = np.exp(log_s)
    I = S * np.exp(np.sum(x * xbar) - 0.5 * np.sum(xbar * xbar))
    theta = float(np.angle(S))
    proj = max(0.0, np.cos(theta))
    e_t = ham.e_trial if e_shift is None else float(e_shift)
    new_w = weight * abs(I) * proj * np.exp(-ham.dt * (ham.const - e_t))
    if proj == 0.0:
        flags |= W_DEAD
    if flags & W_NONFINITE:
        new_w = 0.0
    return {"phi": phi3, "weight": float(new_w), "logo": logo1, "flags": flags,
            "xbar": xbar, "S": S, "I": I, "theta": theta}


def propagate(ham: OracleHamiltonian, phis, weights, logos, x, fb_cap=1.0, taylor_order=6, e_shift=None):
    """One time step for every walker.  x: [W, G] real fields.
    Returns new (phis, weights, logos, flags)."""
    W = phis.shape[0]
    out_phi = np.empty_like(phis)
    out_w = np.empty(W)
    out_l = np.empty(W, dtype=np.complex128)
    flags = np.zeros(W, dtype=np.uint32)
    for w in range(W):
        r = step_walker(ham, phis[w], weights[w], x[w], fb_cap, taylor_order, e_shift)
        out_phi[w], out_w[w], out_l[w], flags[w] = r["phi"], r["weight"], r["logo"], r["flags"]
    return out_phi, out_w, out_l, flags


# ---- re-orthogonalisation --------------------------------------------------------

def mgs(a: np.ndarray):
    """Modified Gram-Schmidt a = Q R with R upper triangular, R_ii > 0."""
    m, n = a.shape
    q = a.astype(np.complex128).copy()
    r = np.zeros((n, n), dtype=np.complex128)
    for k in range(n):
        nrm = np.sqrt(np.sum(np.abs(q[:, k]) ** 2))
        r[k, k] = nrm
        q[:, k] = q[:, k] / nrm
        for j in range(k + 1, n):
            r[k, j] = np.vdot(q[:, k], q[:, j])
            q[:, j] = q[:, j] - r[k, j] * q[:, k]
    return q, r


def reorthogonalize(ham: OracleHamiltonian, phis, logos):
    """phi_s <- Q_s for each spin block; logO -= sum_s sum_i log R_ii."""
    phis = phis.copy()
    logos = np.array(logos, dtype=np.complex128).copy()
    for w in range(phis.shape[0]):
        for sl in ham.spins():
            if sl.stop == sl.start:
                continue
            q, r = mgs(phis[w][:, sl])
            phis[w][:, sl] = q
            logos[w] -= np.sum(np.log(np.diag(r).real))
    return phis, logos


# ---- free projection ---------------------------------------------------------------

def wrap_phase(t: float) -> float:
    """The angle t mapped to (-pi, pi]."""
    return float(np.angle(np.exp(1j * t)))


def free_step_walker(ham: OracleHamiltonian, phi, logo, log_amp, x, taylor_order=6):
    """One free-projection step of one walker (the fp-AFQMC section, reading
    R12): phi' = B(x) phi with the mean-field-shifted propagator of eq. Bprop
    and no force bias; a' = a + log S - dt (C - E_T), with S the overlap ratio of
    eq. ovlp_ratio (its scalar exp(i sqrt(dt) x.l) included).  `logo` is
    log<Psi_T|phi> of the walker as carried.  Returns a dict with the new phi,
    logo, log-amplitude and flags; a walker whose new overlap vanishes keeps
    its logo and amplitude and is flagged singular."""
    flags = 0
    x = np.asarray(x, dtype=float)
    if not np.all(np.isfinite(x)):
        flags |= W_NONFINITE
        x = np.zeros_like(x)
    phi3, logo1, log_s, sing1 = overlap_ratio(ham, phi, logo, x + 0j, taylor_order)
    if sing1:
        return {"phi": phi3, "logo": logo, "log_amp": log_amp, "flags": flags | W_SINGULAR}
    a = log_amp + log_s - ham.dt * (ham.const - ham.e_trial)
    a = complex(a.real, wrap_phase(a.imag))
    return {"phi": phi3, "logo": logo1, "log_amp": a, "flags": flags}


def free_propagate(ham: OracleHamiltonian, phis, logos, amps, x, taylor_order=6):
    """One free-projection step for every walker.  x: [W, G] real fields.
    Returns new (phis, logos, amps, flags)."""
    W = phis.shape[0]
    out_phi = np.empty_like(phis)
    out_l = np.empty(W, dtype=np.complex128)
    out_a = np.empty(W, dtype=np.complex128)
    flags = np.zeros(W, dtype=np.uint32)
    for w in range(W):
        r = free_step_walker(ham, phis[w], logos[w], amps[w], x[w], taylor_order)
        out_phi[w], out_l[w], out_a[w], flags[w] = r["phi"], r["logo"], r["log_amp"], r["flags"]
    return out_phi, out_l, out_a, flags


def free_estimator(weights, amps, energies, flags) -> dict:
    """The fp-AFQMC energy estimate of one set of walkers (reading R12):
    sums N = sum w e^{a - r} E, D = sum w e^{a - r}, N1, N2 (with E1, E2) over
    the walkers that count, r = their largest Re a (0 if none), E = N / D."""
    w = np.asarray(weights, dtype=float)
    a = np.asarray(amps, dtype=np.complex128)
    f = np.asarray(flags, dtype=np.int64)
    use = (w > 0) & ((f & (W_SINGULAR | W_NONFINITE)) == 0) & np.isfinite(a)
    if not use.any():
        return {"N": 0j, "D": 0j, "N1": 0j, "N2": 0j, "r": 0.0, "n": 0, "E": complex(np.nan, np.nan)}
    r = float(np.max(a[use].real))
    z = w[use] * np.exp(a[use] - r)
    e = np.asarray(energies)[use]
    out = {"N": complex(np.sum(z * e[:, 0])), "D": complex(np.sum(z)),
           "N1": complex(np.sum(z * e[:, 1])), "N2": complex(np.sum(z * e[:, 2])),
           "r": r, "n": int(use.sum())}
    out["E"] = out["N"] / out["D"]
    return out


def initial_amplitudes(logos) -> np.ndarray:
    """a = log<Psi_T|phi> for walkers that start with c = 1."""
    return np.array(logos, dtype=np.complex128).copy()


# ---- population control ----------------------------------------------------------

def comb(weights, u: float):
    """Population control by a comb (the paper names population control among the
    steps of the simulation loop, Sec. 3.1, without fixing the method; reading R11: the comb of
    Calandra Buonaura and Sorella, 1998).  With cumulative weights C_i (summed in
    walker order) and total Wt, W teeth sit at (u + k) Wt / W, k = 0..W-1, for one
    uniform u in [0, 1); tooth k selects the first walker i with C_i > tooth.
    Returns the parent of every new walker and the new weights, all Wt / W."""
    w = np.asarray(weights, dtype=float)
    W = len(w)
    c = np.cumsum(w)
    total = c[-1]
    if not total > 0.0:
        return np.arange(W), w.copy()
    step = total / W
    parents = np.empty(W, dtype=int)
    i = 0
    for k in range(W):
        tooth = (u + k) * step
        while i < W - 1 and c[i] <= tooth:
            i += 1
        parents[k] = i
    return parents, np.full(W, step)


# ---- step loop -------------------------------------------------------------------

def initial_logo(ham: OracleHamiltonian, phis) -> np.ndarray:
    return np.array([overlap_theta(ham, p)[0] for p in phis], dtype=np.complex128)


def run(ham: OracleHamiltonian, phis, fields, nsteps, reortho_every=5, fb_cap=1.0,
        taylor_order=6, weights=None):
    """Step loop: propagate; every `reortho_every` steps re-orthogonalise;
    then measure the local energy.  `fields` yields x[W,G] per step.
    Returns per-step records (weights, energies, logos, flags, estimator)."""
    W = phis.shape[0]
    w = np.ones(W) if weights is None else np.asarray(weights, float).copy()
    logo = initial_logo(ham, phis)
    recs = []
    for step in range(1, nsteps + 1):
        x = fields.next()
        phis, w, logo, flags = propagate(ham, phis, w, logo, x, fb_cap, taylor_order)
        if reortho_every and step % reortho_every == 0:
            phis, logo = reorthogonalize(ham, phis, logo)
        e = local_energies(ham, phis)
        recs.append({"step": step, "weights": w.copy(), "energies": e, "logo": logo.copy(),
                     "flags": flags, "est": estimator(w, e)})
    return phis, w, logo, recs


def run_blocks(ham: OracleHamiltonian, phis, fields, nblocks, block_steps, offsets=None, reortho_every=5,
               fb_cap=1.0, taylor_order=6, feedback=True, e_shift=None, weights=None):
    """Block loop (reading R13).  Step n = 1, 2, ... (counted over all blocks)
    propagates with fields.next(), re-orthogonalises when n % reortho_every == 0
    and records the estimator of the new walkers; after each block a comb with
    offset offsets[b] (None: no comb) resamples the walkers and, with
    `feedback`, E_T becomes sum ENumer / sum EDenom of the block.
    Returns the final (phis, weights, logos) and per-block records
    {"est": [per-step estimator dicts], "e_shift": E_T used in the block,
     "parents": comb parents or None}."""
    W = phis.shape[0]
    w = np.ones(W) if weights is None else np.asarray(weights, float).copy()
    logo = initial_logo(ham, phis)
    e_t = ham.e_trial if e_shift is None else float(e_shift)
    blocks = []
    n = 0
    for b in range(nblocks):
        ests = []
        used = e_t
        for _ in range(block_steps):
            n += 1
            phis, w, logo, _ = propagate(ham, phis, w, logo, fields.next(), fb_cap, taylor_order, e_t)
            if reortho_every and n % reortho_every == 0:
                phis, logo = reorthogonalize(ham, phis, logo)
            ests.append(estimator(w, local_energies(ham, phis)))
        parents = None
        if offsets is not None:
            parents, w = comb(w, offsets[b])
            phis, logo = phis[parents], logo[parents]
        if feedback:
            num = sum(e["ENumer"] for e in ests)
            den = sum(e["EDenom"] for e in ests)
            if den > 0.0:
                e_t = num / den
        blocks.append({"est": ests, "e_shift": used, "parents": parents})
    return phis, w, logo, blocks
