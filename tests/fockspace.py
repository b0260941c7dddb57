"""Brute-force Fock-space tools for pinning the oracle on tiny systems.

Everything here works on occupation-number bit strings with explicit fermionic
signs and never uses Wick's theorem, Thouless' theorem or the Cholesky algebra,
so it is an independent check of the oracle.

Spin orbitals: alpha orbital p -> index p, beta orbital p -> index M + p.
A basis determinant |D> = a+_{i1} a+_{i2} ... a+_{iN} |0> with i1 < i2 < ... .
"""
from __future__ import annotations

import itertools

import numpy as np
import scipy.linalg


class FockSector:
    """Determinants with fixed (N_alpha, N_beta) over M spatial orbitals."""

    def __init__(self, m: int, na: int, nb: int):
        self.m, self.na, self.nb = m, na, nb
        dets = []
        for occa in itertools.combinations(range(m), na):
            for occb in itertools.combinations(range(m), nb):
                bits = 0
                for p in occa:
                    bits |= 1 << p
                for p in occb:
                    bits |= 1 << (m + p)
                dets.append(bits)
        self.dets = dets
        self.index = {d: k for k, d in enumerate(dets)}
        self.dim = len(dets)

    # -- single operators on bit strings ------------------------------------------
    @staticmethod
    def annihilate(bits: int, j: int):
        if not (bits >> j) & 1:
            return None, 0
        sign = -1 if bin(bits & ((1 << j) - 1)).count("1") % 2 else 1
        return bits & ~(1 << j), sign

    @staticmethod
    def create(bits: int, j: int):
        if (bits >> j) & 1:
            return None, 0
        sign = -1 if bin(bits & ((1 << j) - 1)).count("1") % 2 else 1
        return bits | (1 << j), sign

    def apply_string(self, bits: int, ops):
        """Apply ops (rightmost first) given as [(dagger, index), ...] written
        left to right as in the operator product.  Returns (bits, sign)."""
        sign = 1
        for dag, j in reversed(ops):
            bits, s = (self.create if dag else self.annihilate)(bits, j)
            if bits is None:
                return None, 0
            sign *= s
        return bits, sign

    # -- operators as dense matrices within the sector -----------------------------------
    def one_body(self, A: np.ndarray) -> np.ndarray:
        """sum_{pq, spin} A_pq a+_{p s} a_{q s} as a dense matrix."""
        m = self.m
        H = np.zeros((self.dim, self.dim), dtype=np.result_type(A, float))
        for k, d in enumerate(self.dets):
            for s in range(2):
                for p in range(m):
                    for q in range(m):
                        if A[p, q] == 0:
                            continue
                        nb, sg = self.apply_string(d, [(1, s * m + p), (0, s * m + q)])
                        if nb is not None:
                            H[self.index[nb], k] += sg * A[p, q]
        return H

    def hamiltonian(self, h: np.ndarray, eri: np.ndarray, ecore: float) -> np.ndarray:
        """H = ecore + sum h_pq a+a + 1/2 sum_{pqrs} sum_{s t} (ps|qr)
        a+_{p s} a+_{q t} a_{r t} a_{s s}, eri[p,s,q,r] = (ps|qr)."""
        m = self.m
        H = self.one_body(h) + ecore * np.eye(self.dim)
        for k, d in enumerate(self.dets):
            for sg1 in range(2):
                for sg2 in range(2):
                    for p, q, r, s in itertools.product(range(m), repeat=4):
                        v = eri[p, s, q, r]
                        if v == 0:
                            continue
                        ops = [(1, sg1 * m + p), (1, sg2 * m + q), (0, sg2 * m + r), (0, sg1 * m + s)]
                        nb, sg = self.apply_string(d, ops)
                        if nb is not None:
                            H[self.index[nb], k] += 0.5 * sg * v
        return H

    # -- Slater determinants ---------------------------------------------------------------
    def slater(self, phi: np.ndarray, na: int) -> np.ndarray:
        """Coefficients of prod_k (sum_p phi~_pk a+_p)|0> where phi~ is the
        2M x (Na+Nb) spin-orbital matrix with phi's alpha columns on the alpha
        orbitals and beta columns on the beta orbitals."""
        m = self.m
        ntot = phi.shape[1]
        big = np.zeros((2 * m, ntot), dtype=np.result_type(phi, float))
        big[:m, :na] = phi[:, :na]
        big[m:, na:] = phi[:, na:]
        c = np.zeros(self.dim, dtype=big.dtype)
        for k, d in enumerate(self.dets):
            occ = [j for j in range(2 * m) if (d >> j) & 1]
            c[k] = np.linalg.det(big[occ, :])
        return c


def eri_from_chol(chol: np.ndarray) -> np.ndarray:
    """(ps|qr) = sum_g L^g_ps L^g_qr as eri[p,s,q,r]."""
    return np.einsum("gps,gqr->psqr", chol, chol)


def expm_dense(H: np.ndarray, t: complex) -> np.ndarray:
    return scipy.linalg.expm(t * H)
