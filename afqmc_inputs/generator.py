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


def make_hamiltonian(spec: SystemSpec):
    """Return (h1 [M,M], chol [Nchol,M,M], ecore) as float64 numpy arrays."""
    rng = np.random.default_rng(spec.seed)
    h1 = make_h1(rng, spec.nbasis)
    chol = make_chol(rng, spec.nbasis, spec.nchol, spec.tau, spec.scale_factor())
    return h1, chol, float(spec.ecore)


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
    trial = make_trial(h1, chol, spec.nalpha, spec.nbeta)
    return h1, chol, ecore, trial


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
                        SystemSpec(1512, 42, 42, 6000, tau=0.75 * 1512), nwalkers=64, nsteps=20)


def batching_specs() -> list[RunSpec]:
    """Sixteen uneven systems: M = 60, 80, ..., 360; N = M/10; Nchol = 4M."""
    counts = batching_walker_counts()
    out = []
    for k, m in enumerate(range(60, 361, 20)):
        n = m // 10
        out.append(RunSpec(f"batch{k}-M{m}", SystemSpec(m, n, n, 4 * m, tau=0.75 * m, seed=100 + k),
                           nwalkers=counts[k]))
    return out
