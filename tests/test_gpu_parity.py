"""Parity of the HIP path (through the C ABI) with the CPU oracle.

FP64 bar: per-walker energies, weights and log-overlaps agree to 1e-10
relative (absolute below magnitude 1), on identical seeded inputs and fields.
"""
import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from pairs import Pair, cmp_rel, phase_diff

pytestmark = pytest.mark.gpu
TOL = 1e-10

RAGGED = gi.SystemSpec(37, 5, 3, 70, tau=30.0, scale="inv_sqrt_m", seed=7)   # open shell, ragged tiles
TILED = gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11)                    # several 64-tiles + tail


def uhf_trial(spec, seed=3):
    h1, chol, _, tr = gi.make_system(spec)
    rng = np.random.default_rng(seed)
    qb, _ = np.linalg.qr(tr[:, spec.nalpha:] + 0.3 * rng.standard_normal((spec.nbasis, spec.nbeta)))
    return np.hstack([tr[:, :spec.nalpha], qb])


@pytest.fixture(scope="module")
def small():
    p = Pair(gi.SMALL.system, gi.SMALL.nwalkers, gi.SMALL.dt)
    yield p
    p.close()


@pytest.fixture(scope="module")
def ragged():
    p = Pair(RAGGED, 7, 0.01, trial=uhf_trial(RAGGED))
    yield p
    p.close()


def test_setup_scalars(small, ragged):
    for p in (small, ragged):
        info = p.A.get_info(p.ctx)
        assert abs(info.e_hf - p.ham.e_trial) < 1e-12 * abs(p.ham.e_trial)
        assert abs(info.const_c - p.ham.const) < 1e-12 * max(1.0, abs(p.ham.const))
        assert info.e_shift == info.e_hf


@pytest.mark.parametrize("which", ["small", "ragged"])
def test_overlap_theta_force_bias(which, small, ragged):
    p = small if which == "small" else ragged
    phis = gi.initial_walkers(p.trial, p.W, noise=0.1, seed=5)
    w = p.walkers(phis)
    th = p.torch.empty_like(w.phi)
    vb = p.torch.empty((p.W, p.ham.nchol), dtype=p.torch.complex128, device="cuda")
    p.A.greens_function(p.ctx, w, th)
    p.A.force_bias(p.ctx, w, vb)
    _, _, logo, flags = p.to_host(w)
    th, vb = th.cpu().numpy(), vb.cpu().numpy()
    assert not flags.any()
    for k in range(p.W):
        lo, thetas, _ = O.overlap_theta(p.ham, phis[k])
        assert phase_diff(logo[k], lo) < TOL
        ref = np.hstack(thetas)
        assert cmp_rel(th[k], ref, np.max(np.abs(ref))) < 1e-12
        vref = O.force_bias(p.ham, thetas)
        assert cmp_rel(vb[k], vref, np.max(np.abs(vref))) < 1e-12


@pytest.mark.parametrize("which,noise", [("small", 0.0), ("small", 0.2), ("ragged", 0.2)])
def test_local_energy(which, noise, small, ragged):
    p = small if which == "small" else ragged
    phis = gi.initial_walkers(p.trial, p.W, noise=noise, seed=9)
    w = p.walkers(phis)
    e, est = p.energies(w)
    ref = O.local_energies(p.ham, phis)
    assert cmp_rel(e, ref) < TOL
    ref_est = O.estimator(np.ones(p.W), ref)
    assert abs(est[0] - ref_est["ENumer"]) < TOL * abs(ref_est["ENumer"])
    assert est[1] == p.W


def run_both(p, nsteps, phis0, reortho_every=5, seed=0, check=None, fb_cap=1.0):
    """Step the GPU and the oracle side by side on identical fields."""
    fields = gi.FieldStream(seed, p.W, p.ham.nchol)
    w = p.walkers(phis0)
    ophi, ow, ologo = phis0.copy(), np.ones(p.W), O.initial_logo(p.ham, phis0)
    worst = {"e": 0.0, "w": 0.0, "logo": 0.0, "phi": 0.0}
    acc_flags = np.zeros(p.W, dtype=np.uint32)  # the library ORs flags in; the oracle reports per step
    for step in range(1, nsteps + 1):
        x = fields.next()
        if check is not None:
            x = check(step, x)
        p.propagate(w, x)
        ophi, ow, ologo, oflags = O.propagate(p.ham, ophi, ow, ologo, x, fb_cap=fb_cap)
        if reortho_every and step % reortho_every == 0:
            p.A.reorthogonalize(p.ctx, w)
            ophi, ologo = O.reorthogonalize(p.ham, ophi, ologo)
        e, est = p.energies(w)
        oe = O.local_energies(p.ham, ophi)
        gphi, gw, glogo, gflags = p.to_host(w)
        acc_flags |= oflags
        assert np.array_equal(gflags, acc_flags), (step, gflags, acc_flags)
        worst["e"] = max(worst["e"], cmp_rel(e, oe))
        worst["w"] = max(worst["w"], cmp_rel(gw, ow))
        worst["logo"] = max(worst["logo"], phase_diff(glogo, ologo))
        ok = (acc_flags & O.W_SINGULAR) == 0  # the oracle stops moving a singular walker
        worst["phi"] = max(worst["phi"], cmp_rel(gphi[ok], ophi[ok], np.max(np.abs(ophi))))
    return worst, (gphi, gw, glogo, gflags), (ophi, ow, ologo)


def test_trajectory_small(small):
    """The 20-step workload: M=24, N=4+4, 96 Cholesky vectors, 10 walkers."""
    worst, g, o = run_both(small, 20, gi.initial_walkers(small.trial, small.W))
    assert worst["e"] < TOL and worst["w"] < TOL and worst["logo"] < TOL and worst["phi"] < TOL, worst
    # restricted trial: alpha and beta blocks stay bitwise equal on the device
    assert np.array_equal(g[0][:, :, :4], g[0][:, :, 4:])


def test_trajectory_ragged_open_shell(ragged):
    worst, g, o = run_both(ragged, 8, gi.initial_walkers(ragged.trial, ragged.W, noise=0.05, seed=2),
                           reortho_every=3)
    assert worst["e"] < TOL and worst["w"] < TOL and worst["logo"] < TOL and worst["phi"] < TOL, worst


def test_trajectory_strong_coupling_cap_active():
    """Literal generator scale at the small size with a tight force-bias cap
    (0.03): the cap is active on many fields and the walk is far from the trial."""
    from paper_2406_16238_amd import afqmc as A
    spec = gi.SystemSpec(24, 4, 4, 96, tau=20.0, scale="literal")
    p = Pair(spec, 10, 0.005, options=A.default_options(fb_cap=0.03))
    try:
        phis = gi.initial_walkers(p.trial, 10, noise=0.05, seed=1)
        r = O.step_walker(p.ham, phis[0], 1.0, np.zeros(96), fb_cap=0.0)
        assert np.sum(np.abs(r["xbar"]) > 0.03) >= 3  # the cap bites
        worst, g, o = run_both(p, 6, phis, fb_cap=0.03)
        assert worst["e"] < 1e-9 and worst["w"] < 1e-9 and worst["phi"] < 1e-9, worst
        # the phaseless projection kills walkers here, on both sides alike
        gflags, gw = g[3], g[1]
        dead = (gflags & O.W_DEAD) != 0
        assert dead.any()
        assert np.all(gw[dead] == 0.0) and np.all(o[1][dead] == 0.0)
    finally:
        p.close()


def test_singular_and_nonfinite_walkers(small):
    phis = gi.initial_walkers(small.trial, small.W, noise=0.02, seed=3)
    phis[0][:, 1] = 0.0  # <Psi_T|phi_0> = 0 exactly

    def poison(step, x):
        x = x.copy()
        if step == 2:
            x[3, 17] = np.nan
        return x

    worst, g, o = run_both(small, 4, phis, reortho_every=0, check=poison)
    gphi, gw, glogo, gflags = g
    assert gflags[0] & O.W_SINGULAR and gw[0] == 0.0
    assert gflags[3] & O.W_NONFINITE and gw[3] == 0.0
    live = [k for k in range(small.W) if k not in (0, 3)]
    assert np.all(gw[live] > 0) and np.all(np.isfinite(gphi))
    assert worst["w"] < TOL


def test_tiled_sizes_parity():
    """M=100, G=200, W=70: several 64-wide tiles with ragged tails on every axis."""
    p = Pair(TILED, 70, 0.005)
    try:
        worst, g, o = run_both(p, 3, gi.initial_walkers(p.trial, 70, noise=0.02, seed=4), reortho_every=2)
        assert worst["e"] < TOL and worst["w"] < TOL and worst["logo"] < TOL and worst["phi"] < TOL, worst
    finally:
        p.close()


WIDE = gi.SystemSpec(96, 42, 41, 192, tau=70.0, seed=13)  # 48-row padded spin blocks, 83 columns


@pytest.mark.parametrize("api", ["separate", "step"])
def test_wide_spin_blocks_parity(api):
    """N = 42 + 41 (the benzene-scale electron count): padded spin blocks of 48
    rows in the exchange and the widest Taylor tile, against the oracle."""
    p = Pair(WIDE, 9, 0.005)
    try:
        phis = gi.initial_walkers(p.trial, 9, noise=0.02, seed=4)
        if api == "separate":
            worst, g, o = run_both(p, 3, phis, reortho_every=2)
            assert worst["e"] < TOL and worst["w"] < TOL and worst["logo"] < TOL and worst["phi"] < TOL, worst
            return
        fields = gi.FieldStream(0, 9, WIDE.nchol)
        w = p.walkers(phis)
        e = p.torch.empty((9, 3), dtype=p.torch.complex128, device="cuda")
        ophi, ow, ologo = phis.copy(), np.ones(9), O.initial_logo(p.ham, phis)
        for step in range(1, 4):
            x = fields.next()
            p.A.step(p.ctx, w, p.torch.as_tensor(x, device="cuda"), e, reortho=(step == 2))
            ophi, ow, ologo, _ = O.propagate(p.ham, ophi, ow, ologo, x)
            if step == 2:
                ophi, ologo = O.reorthogonalize(p.ham, ophi, ologo)
        gphi, gw, glogo, _ = p.to_host(w)
        assert cmp_rel(e.cpu().numpy(), O.local_energies(p.ham, ophi)) < TOL
        assert cmp_rel(gw, ow) < TOL and cmp_rel(gphi, ophi, np.abs(ophi).max()) < TOL
    finally:
        p.close()


def test_deterministic_replay(small):
    outs = []
    for _ in range(2):
        fields = gi.FieldStream(5, small.W, small.ham.nchol)
        w = small.walkers(gi.initial_walkers(small.trial, small.W, noise=0.05, seed=8))
        for step in range(3):
            small.propagate(w, fields.next())
        e, est = small.energies(w)
        outs.append((small.to_host(w), e, est))
    (a, ea, sa), (b, eb, sb) = outs
    for u, v in zip(a, b):
        assert np.array_equal(u, v)
    assert np.array_equal(ea, eb) and np.array_equal(sa, sb)


@pytest.mark.parametrize("spec", [gi.MEDIUM, gi.HEADLINE], ids=["medium-M200", "headline-M400"])
def test_full_size_sampled(spec):
    """Full-size workloads in the benchmark's launch configuration: one step and
    one energy evaluation for every walker on the GPU; the oracle recomputes a
    sample of walkers one by one."""
    p = Pair(spec.system, spec.nwalkers, spec.dt)
    try:
        W = spec.nwalkers
        phis = gi.initial_walkers(p.trial, W, noise=0.01, seed=12)
        x = gi.FieldStream(0, W, spec.system.nchol).next()
        w = p.walkers(phis)
        p.propagate(w, x)
        e, est = p.energies(w)
        gphi, gw, glogo, gflags = p.to_host(w)
        assert not gflags.any()
        sample = np.unique(np.linspace(0, W - 1, 6).astype(int))
        logo0 = O.initial_logo(p.ham, phis[sample])
        for j, k in enumerate(sample):
            r = O.step_walker(p.ham, phis[k], 1.0, x[k])
            assert cmp_rel(gphi[k], r["phi"], np.max(np.abs(r["phi"]))) < TOL
            assert cmp_rel(gw[k], r["weight"]) < TOL
            assert phase_diff(glogo[k], r["logo"]) < TOL
            oe = np.array(O.local_energy(p.ham, r["phi"]))
            assert cmp_rel(e[k], oe) < TOL
    finally:
        p.close()


@pytest.mark.parametrize("bits", [1, 2, 3, 4, 8], ids=["valu-exchange", "valu-gemm", "valu-all", "generic-taylor",
                                                       "unpacked-vhs"])
@pytest.mark.parametrize("spec,W", [(RAGGED, 7), (TILED, 70)], ids=["ragged", "tiled"])
def test_valu_kernels_match_oracle(spec, W, bits):
    """The VALU kernels (kept for comparison runs and as the exchange fallback
    where the MFMA tiling does not apply) and the generic MFMA GEMM for the
    Taylor terms (the fallback of the dedicated kernel) stay at parity too;
    reserved[0] selects them."""
    from paper_2406_16238_amd import afqmc as A
    o = A.default_options()
    o.reserved[0] = bits
    p = Pair(spec, W, 0.01, options=o)
    try:
        worst, g, _ = run_both(p, 2, gi.initial_walkers(p.trial, W, noise=0.05, seed=21), reortho_every=0)
        assert worst["e"] < TOL and worst["w"] < TOL and worst["phi"] < TOL, worst
    finally:
        p.close()


@pytest.mark.parametrize("which", ["small", "tiled"])
def test_fused_step_matches_oracle(which, small):
    """afqmc_step (one LU and one force bias per step, Theta and vbias reused
    across the energy and the next propagation) against the oracle's separate
    propagate / re-orthogonalise / energy sequence."""
    p = small if which == "small" else Pair(TILED, 70, 0.005)
    try:
        W = p.W
        phis = gi.initial_walkers(p.trial, W, noise=0.03, seed=17)
        fields = gi.FieldStream(3, W, p.ham.nchol)
        w = p.walkers(phis)
        e = p.torch.empty((W, 3), dtype=p.torch.complex128, device="cuda")
        est = p.torch.empty((1, 4), dtype=p.torch.float64, device="cuda")
        ophi, ow, ologo = phis.copy(), np.ones(W), O.initial_logo(p.ham, phis)
        for step in range(1, 8):
            x = fields.next()
            reo = step % 3 == 0
            p.A.step(p.ctx, w, p.torch.as_tensor(x, device="cuda"), e, est, reortho=reo)
            ophi, ow, ologo, _ = O.propagate(p.ham, ophi, ow, ologo, x)
            if reo:
                ophi, ologo = O.reorthogonalize(p.ham, ophi, ologo)
            oe = O.local_energies(p.ham, ophi)
            gphi, gw, glogo, gflags = p.to_host(w)
            ge = e.cpu().numpy()
            assert cmp_rel(ge, oe) < TOL, step
            assert cmp_rel(gw, ow) < TOL, step
            assert phase_diff(glogo, ologo) < TOL, step
            assert cmp_rel(gphi, ophi, np.max(np.abs(ophi))) < TOL, step
            oest = O.estimator(ow, oe)
            assert abs(est.cpu().numpy()[0, 0] - oest["ENumer"]) < TOL * abs(oest["ENumer"])
    finally:
        if p is not small:
            p.close()


@pytest.mark.parametrize("shape", [1, 2, 3, 4])
@pytest.mark.parametrize("spec,W", [(TILED, 70), (WIDE, 9)], ids=["tiled", "wide"])
def test_taylor_tiles_match_oracle(spec, W, shape):
    """The Taylor kernel's row tiles (reserved[4] = 1: 48 rows, 2: 32 rows; at
    96 columns always 32 rows) at parity too."""
    from paper_2406_16238_amd import afqmc as A
    o = A.default_options()
    o.reserved[4] = shape
    p = Pair(spec, W, 0.01, options=o)
    try:
        assert A.get_info(p.ctx).taylor_tile == shape - 1
        worst, g, _ = run_both(p, 2, gi.initial_walkers(p.trial, W, noise=0.05, seed=21), reortho_every=0)
        assert worst["e"] < TOL and worst["w"] < TOL and worst["phi"] < TOL, worst
    finally:
        p.close()


def test_taylor_row_tiles_agree_bitwise_and_with_four_products():
    """The row tiles change only which workgroup computes a row: every entry
    sums the same terms in the same order, so the walkers agree bit for bit.
    Against four real products per term (the generic GEMM, reserved[0] bit 2)
    on the same fields: the same walkers to rounding."""
    from paper_2406_16238_amd import afqmc as A
    outs = []
    for bits, shape in ((0, 1), (0, 2), (0, 3), (0, 4), (4, 0)):
        o = A.default_options()
        o.reserved[0] = bits
        o.reserved[4] = shape
        p = Pair(TILED, 40, 0.01, options=o)
        try:
            assert A.get_info(p.ctx).taylor_tile == (shape - 1 if bits == 0 else -1)
            phis = gi.initial_walkers(p.trial, 40, noise=0.05, seed=4)
            w = p.walkers(phis)
            fields = gi.FieldStream(6, 40, p.ham.nchol)
            for _ in range(3):
                p.propagate(w, fields.next())
            outs.append(p.to_host(w))
        finally:
            p.close()
    for other in outs[1:-1]:
        for x, y in zip(outs[0], other):
            assert x.tobytes() == y.tobytes()
    (a, wa, la, _), (b, wb, lb, _) = outs[0], outs[-1]
    assert cmp_rel(a, b, np.abs(b).max()) < 1e-13
    assert cmp_rel(wa, wb) < 1e-13
    assert phase_diff(la, lb) < 1e-12


def test_benzene_shape_sampled():
    """The benzene-dimer-scale shape (M=1512 orbitals, N=42+42, counter recipe of
    the Cholesky tensor) at a reduced G=96, 4 walkers, 3 steps with a
    re-orthogonalisation after the second (the Gram-Schmidt kernel for M > 512
    and the long contraction loops), against the oracle at 1e-10."""
    import dataclasses
    spec = dataclasses.replace(gi.BENZENE_SCALE.system, nchol=96)
    p = Pair(spec, 4, gi.BENZENE_SCALE.dt)
    try:
        worst, g, o = run_both(p, 3, gi.initial_walkers(p.trial, 4, noise=0.01, seed=5), reortho_every=2)
        assert worst["e"] < TOL and worst["w"] < TOL and worst["logo"] < TOL and worst["phi"] < TOL, worst
    finally:
        p.close()
