"""The library's host reblocking (afqmc_reblock) against the oracle's, level by
level, on the CPU (the call touches no device), and its argument checks."""
import numpy as np
import pytest
import scipy.signal

from oracle import blocking as B


@pytest.fixture(scope="module")
def A():
    from paper_2406_16238_amd import afqmc
    afqmc.load_library()
    return afqmc


@pytest.mark.parametrize("n,rho,seed", [(2, 0.0, 1), (7, 0.0, 2), (200, 0.5, 3), (4099, 0.9, 4), (1 << 15, 0.95, 5)])
def test_matches_oracle(A, n, rho, seed):
    e = np.random.default_rng(seed).standard_normal(n)
    x = scipy.signal.lfilter([1.0], [1.0, -rho], e) + 3.0
    got, want = A.reblock(x), B.reblock(x)
    assert got["n"] == want["n"]
    assert got["mean"] == pytest.approx(want["mean"], rel=1e-13, abs=1e-13)
    assert got["optimal"] == want["optimal"]
    assert len(got["levels"]) == len(want["levels"])
    for g, w in zip(got["levels"], want["levels"]):
        assert g["n"] == w["n"]
        for key in ("mean", "std_err", "std_err_err"):
            assert g[key] == pytest.approx(w[key], rel=1e-11, abs=1e-14)


def test_argument_errors(A):
    with pytest.raises(A.AfqmcError) as ei:
        A.reblock([1.0])
    assert ei.value.status == A.ERR_ARG
    with pytest.raises(A.AfqmcError):
        A.reblock([1.0, float("nan"), 2.0])
