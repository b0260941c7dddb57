"""Helpers that drive the HIP path and the CPU oracle on the same seeded inputs."""
from __future__ import annotations

import numpy as np

import afqmc_inputs as gi
from oracle import afqmc_oracle as O


def cmp_rel(a, b, scale=None):
    """max |a - b| / max(|b|, scale)."""
    a = np.asarray(a)
    b = np.asarray(b)
    den = np.maximum(np.abs(b), 1.0 if scale is None else scale)
    return float(np.max(np.abs(a - b) / den)) if a.size else 0.0


def phase_diff(a, b):
    """Distance of two complex logarithms modulo 2 pi i."""
    a = np.asarray(a)
    b = np.asarray(b)
    dre = np.abs(a.real - b.real)
    dim = np.abs(np.angle(np.exp(1j * (a.imag - b.imag))))
    return float(np.max(dre + dim)) if a.size else 0.0


class Pair:
    """One system set up on both sides."""

    def __init__(self, spec: gi.SystemSpec, nwalkers: int, dt: float = 0.005, trial=None, options=None,
                 oracle_kw=None):
        import torch
        from paper_2406_16238_amd import afqmc as A
        self.A = A
        self.torch = torch
        self.spec = spec
        h1, chol, ecore, tr = gi.make_system(spec)
        if trial is not None:
            tr = trial
        self.h1, self.chol, self.ecore, self.trial = h1, chol, ecore, tr
        self.W = nwalkers
        self.dt = dt
        self.ham = O.build(h1, chol, ecore, tr, spec.nalpha, spec.nbeta, dt)
        self.ctx = A.setup_hamiltonian(A.SystemInput(h1, chol, ecore, tr, spec.nalpha, spec.nbeta, nwalkers, dt),
                                       options)

    # -- device walkers -------------------------------------------------------------
    def walkers(self, phis: np.ndarray):
        w = self.A.Walkers.from_numpy(phis)
        self.A.overlap(self.ctx, w)
        return w

    def to_host(self, w):
        self.torch.cuda.synchronize()
        return (w.phi.cpu().numpy(), w.weight.cpu().numpy(), w.log_ovlp.cpu().numpy(),
                w.flags.cpu().numpy().astype(np.uint32))

    def energies(self, w):
        e = self.torch.empty((self.W, 3), dtype=self.torch.complex128, device="cuda")
        est = self.torch.empty((1, 4), dtype=self.torch.float64, device="cuda")
        self.A.local_energy(self.ctx, w, e, est)
        self.torch.cuda.synchronize()
        return e.cpu().numpy(), est.cpu().numpy()[0]

    def propagate(self, w, x: np.ndarray):
        xt = self.torch.as_tensor(np.ascontiguousarray(x), device="cuda")
        self.A.propagate(self.ctx, w, xt)

    def close(self):
        self.ctx.close()
