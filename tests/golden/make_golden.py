"""Writes small_trajectory.json: the oracle's 20-step trajectory of the small
workload (M = 24, N = 4 + 4, 96 Cholesky vectors, 10 walkers started at the
trial, dt = 0.005, N(0,1) fields from seed 0, modified Gram-Schmidt every 5th
step, Sec. 2's phaseless step and eq. Eloc).  Per step it stores the four
sums of the mixed estimator and the walkers' weights.  Only the oracle and
the seeded input generator run here; nothing comes from the HIP path.

    python tests/golden/make_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import afqmc_inputs as gi  # noqa: E402
from oracle import afqmc_oracle as O  # noqa: E402

OUT = os.path.join(HERE, "small_trajectory.json")


def trajectory():
    run = gi.SMALL
    s = run.system
    h1, chol, ecore, trial = gi.make_system(s)
    ham = O.build(h1, chol, ecore, trial, s.nalpha, s.nbeta, run.dt)
    phis = gi.initial_walkers(trial, run.nwalkers)
    fields = gi.FieldStream(0, run.nwalkers, s.nchol)
    _, _, _, recs = O.run(ham, phis, fields, run.nsteps, reortho_every=run.reortho_every)
    return {
        "workload": run.name,
        "nsteps": run.nsteps,
        "dt": run.dt,
        "reortho_every": run.reortho_every,
        "field_seed": 0,
        "steps": [{"step": r["step"], "est": r["est"], "weights": [float(v) for v in r["weights"]]} for r in recs],
    }


if __name__ == "__main__":
    with open(OUT, "w") as f:
        json.dump(trajectory(), f, indent=1)
    print(f"wrote {OUT}")
