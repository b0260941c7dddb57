"""Seeded synthetic inputs for the phaseless-AFQMC walker step.

This module only draws random numbers and arranges them into the inputs the
method consumes: a one-body matrix h, Cholesky vectors L^gamma, a
single-determinant trial, initial walkers and the auxiliary fields x.  It holds
none of the method's arithmetic (no overlaps, force bias, propagator or
energies), so both the CPU oracle and the GPU path may import it.

Recipe (the paper measures on real molecules that are not available; these
synthetic systems stand in for them with the same shapes):

* h: a symmetric M x M matrix.  Its strict upper triangle is drawn from
  N(0, 0.1^2) and mirrored; its diagonal is sort(U(-2, 1)) (ascending).
* L^gamma, gamma = 0..Nchol-1: the upper triangle (with diagonal) of an M x M
  N(0, 1) draw, mirrored, times exp(-gamma / tau) times a global scale.  The
  canonical scale is 1/M (``scale="inv_m"``); ``"literal"`` (scale 1) and
  ``"inv_sqrt_m"`` (1/sqrt(M), a strong-coupling stress case) are kept for
  small systems.  With scale 1 the two-body operator grows like M and the
  sixth-order Taylor propagator diverges beyond M ~ 30.
* Draw order: h's normal block, h's diagonal, then L^0, L^1, ... from one
  numpy ``default_rng(seed)``.
* Trial: the lowest N eigenvectors of F = h + sum_gamma L^gamma tr(L^gamma)/M,
  used for both spins (a restricted closed-shell determinant), laid out as
  [M][N_alpha + N_beta] with the alpha columns first.
* Fields: x[step] of shape [W][Nchol], standard normal, from a separate
  ``default_rng(field_seed)`` drawn step by step.

Counter recipe (``recipe="counter"``, for systems whose Cholesky tensor is too
large to draw on the host; the library can generate the same tensor on the
device, bit for bit):

* L^gamma_pq = L^gamma_qp = sqrt(3) (u_{4i} + u_{4i+1} + u_{4i+2} + u_{4i+3} - 2)
  * (exp(-gamma / tau) * scale) for p <= q, i = (gamma M + p) M + q, where u_n =
  (SplitMix64 output n of the stream seeded with ``seed``) >> 11, times 2^-53
  (a uniform on [0, 1) with 53 bits; the sum of four has mean 2 and variance
  1/3, so the bracket has mean 0 and variance 1).  The four uniforms are added
  left to right, then the bracket is multiplied by sqrt(3) and by the per-vector
  factor (computed with the C library's exp).
* h as in the default recipe (from ``default_rng(seed)``); the trial is the
  lowest N eigenvectors of h alone (no pass over L on the host).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np


@dataclasses.dataclass(frozen=True)
class SystemSpec:
    """Shape and seeds of one synthetic Cholesky-factorised system."""

    nbasis: int
    nalpha: int
    nbeta: int
    nchol: int
    tau: float                 # decay length of the Cholesky magnitudes
    scale: str = "inv_m"       # "inv_m" | "literal" | "inv_sqrt_m"
    seed: int = 0              # Hamiltonian seed
    ecore: float = 0.0
    recipe: str = "rng"        # "rng" (numpy default_rng) | "counter" (SplitMix64 counters)

    @property
    def nelec(self) -> int:
        return self.nalpha + self.nbeta

    def scale_factor(self) -> float:
        if self.scale == "inv_m":
            return 1.0 / self.nbasis
        if self.scale == "literal":
            return 1.0
        if self.scale == "inv_sqrt_m":
            return 1.0 / math.sqrt(self.nbasis)
        raise ValueError(f"unknown scale {self.scale!r}")


@dataclasses.dataclass(frozen=True)
class RunSpec:
    """A workload: one system plus walker count, time step and step count."""

    name: str
    system: SystemSpec
    nwalkers: int
    dt: float = 0.005
    nsteps: int = 20
    reortho_every: int = 5
    field_seed: int = 0


def make_h1(rng: np.random.Generator, m: int) -> np.ndarray:
    off = rng.normal(0.0, 0.1, size=(m, m))
    h = np.triu(off, 1)
    h = h + h.T
    diag = np.sort(rng.uniform(-2.0, 1.0, size=m))
    h[np.diag_indices(m)] = diag
    return h


def make_chol(rng: np.random.Generator, m: int, nchol: int, tau: float,
              scale: float, dtype=np.float64) -> np.ndarray:
    chol = np.empty((nchol, m, m), dtype=dtype)
    for g in range(nchol):
        a = rng.normal(0.0, 1.0, size=(m, m))
        sym = np.triu(a) + np.triu(a, 1).T
        chol[g] = sym * (math.exp(-g / tau) * scale)
    return chol


GOLDEN = 0x9E3779B97F4A7C15
_M64 = (1 << 64) - 1


def splitmix64_outputs(seed: int, n: np.ndarray) -> np.ndarray:
    """Outputs n (uint64 array) of the SplitMix64 stream seeded with `seed`
    (Steele, Lea and Flood 2014): state_n = seed + (n + 1) phi64, mixed."""
    with np.errstate(over="ignore"):
        z = np.uint64(seed & _M64) + (n.astype(np.uint64) + np.uint64(1)) * np.uint64(GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def chol_factors(nchol: int, tau: float, scale: float) -> np.ndarray:
    """exp(-gamma / tau) * scale per Cholesky vector, with the C library's exp."""
    return np.array([math.exp(-g / tau) * scale for g in range(nchol)])


def make_chol_counter(seed: int, m: int, nchol: int, tau: float, scale: float,
                      gammas=None) -> np.ndarray:
    """The counter recipe's L^gamma (all, or the listed gammas) as [len, M, M]."""
    gammas = range(nchol) if gammas is None else list(gammas)
    fac = chol_factors(nchol, tau, scale)
    iu = np.triu_indices(m)
    out = np.empty((len(gammas), m, m))
    root3 = math.sqrt(3.0)
    for k, g in enumerate(gammas):
        i = (np.uint64(g) * np.uint64(m) + iu[0].astype(np.uint64)) * np.uint64(m) + iu[1].astype(np.uint64)
        u = [(splitmix64_outputs(seed, np.uint64(4) * i + np.uint64(r)) >> np.uint64(11)).astype(np.float64)
             * 2.0 ** -53 for r in range(4)]
        z = (((u[0] + u[1]) + u[2]) + u[3]) - 2.0
        v = (z * root3) * fac[g]
        out[k][iu] = v
        out[k][(iu[1], iu[0])] = v
    return out


def make_hamiltonian(spec: SystemSpec):
    """Return (h1 [M,M], chol [Nchol,M,M], ecore) as float64 numpy arrays."""
    rng = np.random.default_rng(spec.seed)
    h1 = make_h1(rng, spec.nbasis)
    if spec.recipe == "counter":
        chol = make_chol_counter(spec.seed, spec.nbasis, spec.nchol, spec.tau, spec.scale_factor())
    else:
        chol = make_chol(rng, spec.nbasis, spec.nchol, spec.tau, spec.scale_factor())
    return h1, chol, float(spec.ecore)


def make_h1_only(spec: SystemSpec) -> np.ndarray:
    return make_h1(np.random.default_rng(spec.seed), spec.nbasis)


def make_trial_from_h(h1: np.ndarray, nalpha: int, nbeta: int) -> np.ndarray:
    """Lowest eigenvectors of h alone (the counter recipe's trial)."""
    _, vecs = np.linalg.eigh(0.5 * (h1 + h1.T))
    return np.ascontiguousarray(np.hstack([vecs[:, :nalpha], vecs[:, :nbeta]]))


def make_trial(h1: np.ndarray, chol: np.ndarray, nalpha: int, nbeta: int) -> np.ndarray:
    """Lowest eigenvectors of h + sum_g L^g tr(L^g)/M, alpha block then beta block."""
    m = h1.shape[0]
    tr = np.einsum("gpp->g", chol)
    fock = h1 + np.tensordot(tr, chol, axes=1) / m
    fock = 0.5 * (fock + fock.T)
    _, vecs = np.linalg.eigh(fock)
    orbs_a = vecs[:, :nalpha]
    orbs_b = vecs[:, :nbeta]
    return np.ascontiguousarray(np.hstack([orbs_a, orbs_b]))


def make_system(spec: SystemSpec):
    """Hamiltonian plus trial for one spec."""
    h1, chol, ecore = make_hamiltonian(spec)
    if spec.recipe == "counter":
        trial = make_trial_from_h(h1, spec.nalpha, spec.nbeta)
    else:
        trial = make_trial(h1, chol, spec.nalpha, spec.nbeta)
    return h1, chol, ecore, trial


def make_system_without_chol(spec: SystemSpec):
    """(h1, ecore, trial) of a counter-recipe spec, whose L is generated on the device."""
    if spec.recipe != "counter":
        raise ValueError("only the counter recipe can leave L to the device")
    h1 = make_h1_only(spec)
    return h1, float(spec.ecore), make_trial_from_h(h1, spec.nalpha, spec.nbeta)


def initial_walkers(trial: np.ndarray, nwalkers: int, noise: float = 0.0,
                    seed: int = 1) -> np.ndarray:
    """Walker slab [W][M][N_alpha+N_beta] complex128, equal to the trial plus
    optional complex Gaussian noise of the given standard deviation."""
    phi = np.broadcast_to(trial.astype(np.complex128), (nwalkers,) + trial.shape).copy()
    if noise > 0.0:
        rng = np.random.default_rng(seed)
        phi += noise * (rng.standard_normal(phi.shape) + 1j * rng.standard_normal(phi.shape))
    return phi


class FieldStream:
    """Auxiliary fields x[step] ~ N(0,1), shape [W][Nchol], drawn step by step."""

    def __init__(self, seed: int, nwalkers: int, nchol: int):
        self.rng = np.random.default_rng(seed)
        self.shape = (nwalkers, nchol)
        self.step = 0

    def next(self) -> np.ndarray:
        self.step += 1
        return self.rng.standard_normal(self.shape)


def batching_walker_counts(seed: int = 3, nsys: int = 16) -> list[int]:
    """Walker counts of the multi-system workload: uniform integers in [64, 512]."""
    return [int(v) for v in np.random.default_rng(seed).integers(64, 513, nsys)]


# ---- named workloads ---------------------------------------------------------

SMALL = RunSpec("small-M24-N4-chol96",
                SystemSpec(24, 4, 4, 96, tau=20.0), nwalkers=10, nsteps=20)
MEDIUM = RunSpec("medium-M200-N20-chol800",
                 SystemSpec(200, 20, 20, 800, tau=150.0), nwalkers=512, nsteps=200)
HEADLINE = RunSpec("headline-M400-N40-chol1600",
                   SystemSpec(400, 40, 40, 1600, tau=300.0), nwalkers=256, nsteps=20)
BENZENE_SCALE = RunSpec("benzene-scale-M1512-N42-chol6000",
                        SystemSpec(1512, 42, 42, 6000, tau=0.75 * 1512, recipe="counter"), nwalkers=64, nsteps=20)


def batching_specs() -> list[RunSpec]:
    """Sixteen uneven systems: M = 60, 80, ..., 360; N = M/10; Nchol = 4M."""
    counts = batching_walker_counts()
    out = []
    for k, m in enumerate(range(60, 361, 20)):
        n = m // 10
        out.append(RunSpec(f"batch{k}-M{m}", SystemSpec(m, n, n, 4 * m, tau=0.75 * m, seed=100 + k),
                           nwalkers=counts[k]))
    return out
