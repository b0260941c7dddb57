"""CPU oracle of the learned control-variate form of the exchange energy.

TEST INFRASTRUCTURE ONLY (imported by the tests, the smoke check and the
benchmark's CPU leg; never by the product path).  Plain numpy float64.

The exchange energy EK_w of every walker (the expensive part of the local
energy, eq. Eloc of the paper's theory section) is replaced in the mixed
estimator by a control variate:
  * a small network f predicts EK_w from cheap per-walker features;
  * the exact EK_w is computed on a uniform random subset S of k walkers drawn
    without replacement (inclusion probability pi = k / W for every walker);
  * each walker gets the Horvitz-Thompson estimate
        g_w = f_w + [w in S] (EK_w - f_w) / pi,
    whose expectation over S is EK_w for every walker, so the estimator
    sum_w w_w Re(E1 + EJ + g)_w / sum_w w_w is unbiased given the walker states
    (the weights do not depend on the sampled energies).
Conditional variance of sum_w omega_w g_w (omega = normalised weights, sampling
without replacement): (1/pi - 1) * W/(W-1) * sum_w omega_w^2 d_w^2
- (1/pi - 1)/(W-1) * (sum_w omega_w d_w)^2 with d = EK - f  (finite-population form).

Features: besides the Coulomb energy, the one-body energy, the force-bias
norms and the overlap phase, the first-order exchange: EK(Theta) expanded about
the trial (Theta = Psi) is EK(Psi) - sum_s Tr(K_s (Theta_s - Psi_s)) with
K_s = sum_g (Ltilde^{g s} Psi_s) Ltilde^{g s} (N x M), so Tr(K_s Theta_s) summed
over spins carries the walker's exchange energy to first order at the cost of a
one-body energy.

Network: x (10 features, standardised) -> tanh(W1 x + b1) (128) -> tanh(W2 h + b2)
(128) -> W3 h + b3 (2 outputs: Re and Im of the standardised EK).
Training: mean squared error, Adam (Kingma & Ba 2015: beta1 = 0.9,
beta2 = 0.999, eps = 1e-8, bias-corrected moments).
Subset keys: SplitMix64 (Steele, Lea and Flood, OOPSLA 2014) output function
applied to seed + call * 2^32 + w + 1 times the golden-ratio increment; the k
walkers with the smallest keys (ties to the lower index) form S.
"""
from __future__ import annotations

import numpy as np

NFEAT = 10
HIDDEN = 128
NOUT = 2
MASK64 = (1 << 64) - 1
GOLDEN = 0x9E3779B97F4A7C15


# ---- features --------------------------------------------------------------------

def exchange_first_order_matrices(ham) -> list:
    """K_s = sum_g (Ltilde^{g s} Psi_s) Ltilde^{g s} per spin block (N_s x M)."""
    out = []
    for s, sl in enumerate(ham.spins()):
        lh = ham.lhalf[s]                        # [G, N_s, M]
        t0 = np.matmul(lh, ham.trial[:, sl])     # Ltilde Psi, [G, N_s, N_s]
        out.append(np.einsum("gij,gjq->iq", t0, lh))
    return out


def features(ham, phi, oracle, kmats=None) -> np.ndarray:
    """(Re EJ, Im EJ, Re E1, Im E1, sum|vbias - l|^2, Re sum (vbias - l)^2,
    cos arg<Psi_T|phi>, sin arg<Psi_T|phi>, Re sum_s Tr(K_s Theta_s),
    Im sum_s Tr(K_s Theta_s)) of one walker.  `kmats`: the K_s of
    exchange_first_order_matrices (computed when None)."""
    logo, thetas, _ = oracle.overlap_theta(ham, phi)
    _, e1, _ = oracle.local_energy(ham, phi)
    vb = oracle.force_bias(ham, thetas)
    ej = 0.5 * np.sum(vb * vb)
    d = vb - ham.lmf
    ks = exchange_first_order_matrices(ham) if kmats is None else kmats
    lin = sum(np.einsum("iq,qi->", k, th) for k, th in zip(ks, thetas))
    return np.array([ej.real, ej.imag, e1.real, e1.imag, np.sum(np.abs(d) ** 2), np.sum(d * d).real,
                     np.cos(logo.imag), np.sin(logo.imag), lin.real, lin.imag])


def exchange_energy(ham, phi, oracle) -> complex:
    """EK = E2 - EJ of one walker (the exchange part of the local energy)."""
    _, thetas, _ = oracle.overlap_theta(ham, phi)
    _, _, e2 = oracle.local_energy(ham, phi)
    vb = oracle.force_bias(ham, thetas)
    return e2 - 0.5 * np.sum(vb * vb)


# ---- network ------------------------------------------------------------------------

def init_params(seed: int = 0) -> dict:
    """Glorot-uniform weights, zero biases."""
    rng = np.random.default_rng(seed)

    def glorot(fan_in, fan_out):
        lim = np.sqrt(6.0 / (fan_in + fan_out))
        return rng.uniform(-lim, lim, size=(fan_out, fan_in))

    return {"W1": glorot(NFEAT, HIDDEN), "b1": np.zeros(HIDDEN),
            "W2": glorot(HIDDEN, HIDDEN), "b2": np.zeros(HIDDEN),
            "W3": glorot(HIDDEN, NOUT), "b3": np.zeros(NOUT)}


PARAM_ORDER = ("W1", "b1", "W2", "b2", "W3", "b3")


def flatten(p: dict) -> np.ndarray:
    return np.concatenate([p[k].ravel() for k in PARAM_ORDER])


def unflatten(v: np.ndarray) -> dict:
    shapes = {"W1": (HIDDEN, NFEAT), "b1": (HIDDEN,), "W2": (HIDDEN, HIDDEN), "b2": (HIDDEN,),
              "W3": (NOUT, HIDDEN), "b3": (NOUT,)}
    out, o = {}, 0
    for k in PARAM_ORDER:
        n = int(np.prod(shapes[k]))
        out[k] = np.asarray(v[o:o + n], float).reshape(shapes[k])
        o += n
    return out


def forward(p: dict, X: np.ndarray):
    """X [n, NFEAT] (standardised) -> (Y [n, 2], cache)."""
    z1 = X @ p["W1"].T + p["b1"]
    h1 = np.tanh(z1)
    z2 = h1 @ p["W2"].T + p["b2"]
    h2 = np.tanh(z2)
    y = h2 @ p["W3"].T + p["b3"]
    return y, (X, h1, h2)


def loss_and_grad(p: dict, X: np.ndarray, T: np.ndarray):
    """Mean over samples of 1/2 ||y - t||^2 and its gradient (backpropagation)."""
    y, (X, h1, h2) = forward(p, X)
    n = X.shape[0]
    r = (y - T) / n
    loss = 0.5 * np.sum((y - T) ** 2) / n
    g = {"W3": r.T @ h2, "b3": r.sum(0)}
    d2 = (r @ p["W3"]) * (1.0 - h2 ** 2)
    g["W2"] = d2.T @ h1
    g["b2"] = d2.sum(0)
    d1 = (d2 @ p["W2"]) * (1.0 - h1 ** 2)
    g["W1"] = d1.T @ X
    g["b1"] = d1.sum(0)
    return loss, g


def adam_step(p: dict, g: dict, m: dict, v: dict, t: int, lr: float, b1=0.9, b2=0.999, eps=1e-8):
    """One Adam update (t counts from 1)."""
    for k in PARAM_ORDER:
        m[k] = b1 * m[k] + (1 - b1) * g[k]
        v[k] = b2 * v[k] + (1 - b2) * g[k] ** 2
        mh = m[k] / (1 - b1 ** t)
        vh = v[k] / (1 - b2 ** t)
        p[k] = p[k] - lr * mh / (np.sqrt(vh) + eps)


# ---- subset and estimator ---------------------------------------------------------

def splitmix64(x: int) -> int:
    """SplitMix64 output for state x (the state is advanced by GOLDEN first)."""
    z = (x + GOLDEN) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def subset(seed: int, call: int, W: int, k: int) -> np.ndarray:
    """Indices of the k walkers with the smallest keys (ties: lower index)."""
    keys = [splitmix64((seed + (call << 32) + w * GOLDEN) & MASK64) for w in range(W)]
    order = sorted(range(W), key=lambda w: (keys[w], w))
    return np.array(sorted(order[:k]), dtype=int)


def ht_exchange(f: np.ndarray, ek: np.ndarray, S, pi: float) -> np.ndarray:
    """Per-walker Horvitz-Thompson estimates g_w = f_w + [w in S](EK_w - f_w)/pi."""
    g = np.array(f, dtype=complex)
    for w in S:
        g[w] = f[w] + (ek[w] - f[w]) / pi
    return g


def cv_variance(omega: np.ndarray, d: np.ndarray, pi: float) -> float:
    """Variance over S of sum_w omega_w g_w for real residuals d = EK - f."""
    W = len(omega)
    a = omega * d
    return (1 / pi - 1) * (W / (W - 1) * np.sum(a ** 2) - np.sum(a) ** 2 / (W - 1))
