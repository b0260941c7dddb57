"""Population control (comb) and the energy-shift setter, through the C ABI,
against the oracle's comb (pinned on the CPU: copies floor/ceil of W w / Wt,
total weight kept, exact expectation over the offset)."""
import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from pairs import Pair, cmp_rel, phase_diff

pytestmark = pytest.mark.gpu
TOL = 1e-10


def test_comb_matches_oracle():
    spec = gi.SystemSpec(40, 5, 4, 80, tau=30.0, seed=3)
    W = 45
    p = Pair(spec, W, 0.005)
    A, torch = p.A, p.torch
    try:
        phis = gi.initial_walkers(p.trial, W, noise=0.05, seed=2)
        w = p.walkers(phis)
        rng = np.random.default_rng(6)
        wt = rng.exponential(1.0, W)
        wt[[0, 7, 44]] = 0.0
        w.weight.copy_(torch.as_tensor(wt))
        w.flags.copy_(torch.as_tensor(np.arange(W, dtype=np.int32)))   # tags to follow the copies
        logo_before = w.log_ovlp.cpu().numpy()
        u = 0.3711
        parents = torch.empty(W, dtype=torch.int32, device="cuda")
        A.population_control(p.ctx, w, torch.tensor([u], dtype=torch.float64, device="cuda"), parents)
        torch.cuda.synchronize()
        op, ow = O.comb(wt, u)
        gpar = parents.cpu().numpy()
        assert np.array_equal(gpar, op)
        assert w.weight.cpu().numpy().tobytes() == ow.tobytes()
        assert np.array_equal(w.phi.cpu().numpy(), phis[op])
        assert np.array_equal(w.log_ovlp.cpu().numpy(), logo_before[op])
        assert np.array_equal(w.flags.cpu().numpy(), op.astype(np.int32))
        assert not np.isin([0, 7, 44], op).any()
    finally:
        p.close()


def test_trajectory_with_population_control():
    """Steps with a comb every 4 steps, against the oracle doing the same."""
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        W = p.W
        phis = gi.initial_walkers(p.trial, W, noise=0.05, seed=9)
        fields = gi.FieldStream(4, W, p.ham.nchol)
        us = np.random.default_rng(12).random(4)
        w = p.walkers(phis)
        e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        ophi, ow, ologo = phis.copy(), np.ones(W), O.initial_logo(p.ham, phis)
        worst = 0.0
        for step in range(1, 13):
            x = fields.next()
            A.step(p.ctx, w, torch.as_tensor(x, device="cuda"), e, reortho=(step % 5 == 0))
            ophi, ow, ologo, _ = O.propagate(p.ham, ophi, ow, ologo, x)
            if step % 5 == 0:
                ophi, ologo = O.reorthogonalize(p.ham, ophi, ologo)
            if step % 4 == 0:
                u = us[step // 4 - 1]
                A.population_control(p.ctx, w, torch.tensor([u], dtype=torch.float64, device="cuda"))
                par, ow = O.comb(ow, u)
                ophi, ologo = ophi[par], ologo[par]
            torch.cuda.synchronize()
            gphi, gw, glogo, _ = p.to_host(w)
            worst = max(worst, cmp_rel(gw, ow), cmp_rel(gphi, ophi, np.abs(ophi).max()), phase_diff(glogo, ologo))
        # the energies of the final, resampled walkers
        e2 = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        A.local_energy(p.ctx, w, e2)
        worst = max(worst, cmp_rel(e2.cpu().numpy(), O.local_energies(p.ham, ophi)))
        assert worst < TOL, worst
    finally:
        p.close()


def test_set_e_shift_scales_the_weights():
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        phis = gi.initial_walkers(p.trial, 10, noise=0.02, seed=3)
        x = gi.FieldStream(1, 10, p.ham.nchol).next()
        e = torch.empty((10, 3), dtype=torch.complex128, device="cuda")
        out = []
        base = A.get_info(p.ctx, 0).e_shift
        for shift in (base, base + 0.25):
            A.set_e_shift(p.ctx, shift)
            assert A.get_info(p.ctx, 0).e_shift == shift
            w = p.walkers(phis)
            A.step(p.ctx, w, torch.as_tensor(x, device="cuda"), e, fresh=True)
            torch.cuda.synchronize()
            out.append(w.weight.cpu().numpy())
        assert np.allclose(out[1] / out[0], np.exp(0.005 * 0.25), rtol=1e-13, atol=0)
    finally:
        p.close()
