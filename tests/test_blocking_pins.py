"""Pins of the oracle's reblocking analysis (oracle/blocking.py) against values
fixed by hand, by the closed-form variance of the mean of an AR(1) process,
and by the coverage of its error bars over many independent series."""
import numpy as np
import pytest
import scipy.signal

from oracle import blocking as B


def test_levels_by_hand():
    # level 0: mean 3, c0 = 32/8 = 4; level 1: (2, 4, 5, 1), c0 = 10/4;
    # level 2: (3, 3), c0 = 0; a single sample ends the levels
    lv = B.block_levels([1, 3, 2, 6, 5, 5, 0, 2])
    assert [v["n"] for v in lv] == [8, 4, 2]
    assert [v["mean"] for v in lv] == [3.0, 3.0, 3.0]
    assert lv[0]["std_err"] == pytest.approx(np.sqrt(4.0 / 7.0), rel=1e-15)
    assert lv[1]["std_err"] == pytest.approx(np.sqrt(2.5 / 3.0), rel=1e-15)
    assert lv[2]["std_err"] == 0.0
    assert lv[0]["std_err_err"] == pytest.approx(np.sqrt(4.0 / 7.0) / np.sqrt(14.0), rel=1e-15)


def test_odd_sample_dropped_at_each_level():
    # 7 samples: level 1 pairs (1,2), (3,4), (5,6) and drops 7; level 2 keeps (1.5, 3.5)
    lv = B.block_levels([1, 2, 3, 4, 5, 6, 7])
    assert [v["n"] for v in lv] == [7, 3]
    assert lv[1]["mean"] == pytest.approx(3.5, rel=1e-15)
    assert lv[1]["std_err"] == pytest.approx(np.sqrt((4.0 + 0.0 + 4.0) / 3.0 / 2.0), rel=1e-15)
    assert len(B.block_levels([1.0])) == 0


def test_optimal_level_rule():
    # e_B / e_0 = 1, 2, 3, 3, ...: 2^(3B) > 2 * 1000 * 81 first at B = 6; the same
    # rule with the ratio squared instead of to the fourth power would stop at B = 5
    levels = [{"level": b, "std_err": [1.0, 2.0, 3.0][min(b, 2)]} for b in range(9)]
    assert B.optimal_level(levels, 1000) == 6
    assert B.optimal_level(levels[:6], 1000) is None


def _ar1(rng, rho, n, count):
    e = rng.standard_normal((count, n))
    e[:, 0] /= np.sqrt(1.0 - rho * rho)      # stationary start
    return scipy.signal.lfilter([np.sqrt(1.0 - rho * rho)], [1.0, -rho], e, axis=1)


def _ar1_var_of_mean(rho, n):
    # (1/n^2) sum_{i,j} rho^|i-j| in closed form
    return ((1.0 + rho) / (1.0 - rho) - 2.0 * rho * (1.0 - rho ** n) / (n * (1.0 - rho) ** 2)) / n


def test_uncorrelated_series():
    x = np.random.default_rng(11).standard_normal(1 << 14)
    r = B.reblock(x)
    assert r["levels"][0]["std_err"] == pytest.approx(np.std(x, ddof=1) / np.sqrt(x.size), rel=1e-12)
    assert r["optimal"] is not None
    assert r["std_err"] == pytest.approx(1.0 / np.sqrt(x.size), rel=0.15)


def test_ar1_error_bar_matches_closed_form():
    rho, n = 0.9, 1 << 16
    x = _ar1(np.random.default_rng(5), rho, n, 1)[0]
    r = B.reblock(x)
    exact = np.sqrt(_ar1_var_of_mean(rho, n))
    assert r["optimal"] is not None and r["optimal"] >= 4
    lv = r["levels"][r["optimal"]]
    assert abs(r["std_err"] - exact) < 3.0 * lv["std_err_err"] + 0.02 * exact
    # level 0 (no blocking) underestimates by about sqrt((1 + rho) / (1 - rho))
    assert r["levels"][0]["std_err"] < 0.3 * exact


def test_ar1_coverage_over_many_series():
    rho, n, count = 0.8, 4096, 400
    xs = _ar1(np.random.default_rng(8), rho, n, count)
    exact = _ar1_var_of_mean(rho, n)
    inside, var_est = 0, []
    for x in xs:
        r = B.reblock(x)
        assert r["optimal"] is not None
        var_est.append(r["std_err"] ** 2)
        inside += abs(r["mean"]) < 2.0 * r["std_err"]
    # the estimated variance of the mean averages to the exact one, and the
    # two-sigma intervals cover the true mean (0) about 95 % of the time
    assert np.mean(var_est) == pytest.approx(exact, rel=0.1)
    assert 0.90 <= inside / count <= 0.99
