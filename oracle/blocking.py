"""Reblocking analysis of a serially correlated series (oracle side).

TEST INFRASTRUCTURE ONLY.  Only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this module.

The paper's driver writes its estimates once per block so that they can be
reblocked while the run goes on (Sec. 3.1, citing Flyvbjerg and Petersen).  It
does not spell the analysis out; this module writes it down from the two
published sources it rests on:

* H. Flyvbjerg and H. G. Petersen, J. Chem. Phys. 91, 461 (1989): for samples
  x_1..x_n with mean m and c0 = (1/n) sum (x_i - m)^2, the variance of m is
  bounded below by c0 / (n - 1), with equality for uncorrelated samples.  The
  blocking transformation x'_i = (x_{2i-1} + x_{2i}) / 2 (n' = floor(n / 2),
  an odd last sample dropped) leaves the variance of the mean unchanged while
  the bound rises towards it; the estimate at each level carries the relative
  error 1 / sqrt(2 (n - 1)).
* R. M. Lee, G. J. Conduit, N. Nemec, P. Lopez Rios and N. D. Drummond,
  Phys. Rev. E 83, 066706 (2011): the level B to read off is the smallest one
  whose block length 2^B satisfies 2^(3B) > 2 n0 (e_B / e_0)^4, e_B the
  standard error estimated at level B and n0 the number of original samples.

Plain Python/numpy in float64, one level at a time.
"""
from __future__ import annotations

import numpy as np


def block_levels(x):
    """Every blocking level with at least two samples.

    Returns a list of dicts, level 0 first: {"level", "n", "mean",
    "std_err" = sqrt(c0 / (n - 1)), "std_err_err" = std_err / sqrt(2 (n - 1))}."""
    data = np.asarray(x, dtype=np.float64).ravel()
    levels = []
    lev = 0
    while data.size >= 2:
        n = data.size
        m = float(np.mean(data))
        c0 = float(np.sum((data - m) ** 2)) / n
        se = float(np.sqrt(c0 / (n - 1)))
        levels.append({"level": lev, "n": n, "mean": m, "std_err": se,
                       "std_err_err": se / float(np.sqrt(2.0 * (n - 1)))})
        half = n // 2
        data = 0.5 * (data[0:2 * half:2] + data[1:2 * half:2])
        lev += 1
    return levels


def optimal_level(levels, n0):
    """The Lee et al. choice: the smallest level B with 2^(3B) > 2 n0 (e_B/e_0)^4;
    None when no level qualifies (the series is too short for its correlation)."""
    if not levels:
        return None
    e0 = levels[0]["std_err"]
    for lv in levels:
        b = lv["level"]
        ratio4 = (lv["std_err"] / e0) ** 4 if e0 > 0.0 else 1.0
        if 2.0 ** (3 * b) > 2.0 * n0 * ratio4:
            return b
    return None


def reblock(x):
    """Mean of the series, its standard error at the optimal level (None when
    no level qualifies) and every level's figures."""
    data = np.asarray(x, dtype=np.float64).ravel()
    levels = block_levels(data)
    opt = optimal_level(levels, data.size)
    return {"n": int(data.size), "mean": float(np.mean(data)) if data.size else float("nan"),
            "optimal": opt, "std_err": levels[opt]["std_err"] if opt is not None else None,
            "levels": levels}
