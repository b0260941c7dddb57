"""The stored oracle trajectory of the small workload (tests/golden/
small_trajectory.json, written by tests/golden/make_golden.py from the oracle
alone): the oracle still reproduces it, its records are self-consistent, and
the HIP path (through the C ABI, on the GPU) reproduces it step by step."""
import json
import os

import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "small_trajectory.json")
TOL = 1e-10


def _golden():
    with open(GOLDEN) as f:
        return json.load(f)


def _rel(a, b):
    return abs(a - b) / max(abs(b), 1e-300)


def test_golden_records_are_self_consistent():
    g = _golden()
    run = gi.SMALL
    assert g["workload"] == run.name and g["nsteps"] == run.nsteps == len(g["steps"])
    assert g["dt"] == run.dt and g["reortho_every"] == run.reortho_every
    for rec in g["steps"]:
        est, w = rec["est"], np.array(rec["weights"])
        assert len(w) == run.nwalkers and np.all(w >= 0)
        assert abs(est["EDenom"] - w.sum()) < 1e-12 * w.sum()
        assert abs(est["ENumer"] - est["E1Body"] - est["E2Body"]) < 1e-10 * abs(est["ENumer"])


def test_oracle_reproduces_golden_trajectory():
    import importlib.util
    spec = importlib.util.spec_from_file_location("make_golden", os.path.join(os.path.dirname(GOLDEN), "make_golden.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    now, g = mod.trajectory(), _golden()
    for a, b in zip(now["steps"], g["steps"]):
        for k in ("ENumer", "EDenom", "E1Body", "E2Body"):
            assert _rel(a["est"][k], b["est"][k]) < TOL, (a["step"], k)
        assert np.max(np.abs(np.array(a["weights"]) - np.array(b["weights"]))) < TOL


@pytest.mark.gpu
def test_hip_path_reproduces_golden_trajectory():
    from pairs import Pair
    g = _golden()
    run = gi.SMALL
    p = Pair(run.system, run.nwalkers, run.dt)
    try:
        w = p.walkers(gi.initial_walkers(p.trial, run.nwalkers))
        fields = gi.FieldStream(g["field_seed"], run.nwalkers, run.system.nchol)
        for rec in g["steps"]:
            p.propagate(w, fields.next())
            if rec["step"] % g["reortho_every"] == 0:
                p.A.reorthogonalize(p.ctx, w)
            _, est = p.energies(w)
            for k, v in zip(("ENumer", "EDenom", "E1Body", "E2Body"), est):
                assert _rel(v, rec["est"][k]) < TOL, (rec["step"], k, v, rec["est"][k])
            _, gw, _, _ = p.to_host(w)
            assert np.max(np.abs(gw - np.array(rec["weights"]))) < TOL, rec["step"]
    finally:
        p.close()
