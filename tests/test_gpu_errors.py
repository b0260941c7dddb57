"""Forced failures and cache hazards through the C ABI: the device-memory
limit of set-up (nothing stays allocated), and new walkers that reuse the
device addresses of the previous step's walkers."""
import numpy as np
import pytest

import afqmc_inputs as gi
from oracle import afqmc_oracle as O
from pairs import Pair, cmp_rel, phase_diff

pytestmark = pytest.mark.gpu


def test_mem_limit_refuses_setup_and_frees_everything():
    import torch
    from paper_2406_16238_amd import afqmc as A
    specs = [gi.SystemSpec(100, 10, 10, 200, tau=75.0, seed=11), gi.SystemSpec(120, 12, 12, 240, tau=90.0, seed=12)]
    inputs = []
    for sp in specs:
        h1, chol, ecore, trial = gi.make_system(sp)
        inputs.append(A.SystemInput(h1, chol, ecore, trial, sp.nalpha, sp.nbeta, 64, 0.005))
    torch.cuda.synchronize()
    one = A.setup_hamiltonian(inputs[0])
    need0 = A.get_info(one, 0).device_bytes
    one.close()
    torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    # a limit below the first system: refused before any allocation; a limit
    # that fits the first system (its buffers, the full Cholesky tensor it holds
    # until set-up ends, and its set-up temporaries) but not the second: refused
    # after the first system was allocated, and everything is freed again
    M0, G0, Nt0 = specs[0].nbasis, specs[0].nchol, specs[0].nalpha + specs[0].nbeta
    fits_first = need0 + 8 * G0 * M0 * M0 + 8 * (69 * M0 * M0 + G0) + 16 * (M0 * Nt0 + 3) + (1 << 20)
    for limit in (1 << 20, fits_first):
        with pytest.raises(A.AfqmcError) as ei:
            A.setup_hamiltonian(inputs, A.default_options(mem_limit_bytes=limit))
        assert ei.value.status == A.ERR_OOM
        assert "mem_limit_bytes" in str(ei.value)
        torch.cuda.synchronize()
        free1, _ = torch.cuda.mem_get_info()
        assert abs(free1 - free0) < (8 << 20), (limit, free0 - free1)
    # the library still works afterwards
    ctx = A.setup_hamiltonian(inputs, A.default_options(mem_limit_bytes=1 << 40))
    ctx.close()


def test_new_walkers_at_old_addresses_are_recomputed():
    """A step, then fresh walker tensors that the caching allocator places at
    the freed tensors' addresses, with log<Psi_T|phi> filled by the caller (no
    library call in between): the step must not reuse the old walkers' Green's
    function."""
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        W, G = p.W, p.ham.nchol
        e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
        fs = gi.FieldStream(2, W, G)
        x = torch.empty((W, G), dtype=torch.float64, device="cuda")
        old = p.walkers(gi.initial_walkers(p.trial, W, noise=0.05, seed=1))
        x.copy_(torch.as_tensor(fs.next()))
        A.step(p.ctx, old, x, e)
        torch.cuda.synchronize()
        addr = old.phi.data_ptr()
        del old
        phis = gi.initial_walkers(p.trial, W, noise=0.05, seed=2)
        new = A.Walkers.from_numpy(phis)
        new.log_ovlp.copy_(torch.as_tensor(O.initial_logo(p.ham, phis)))
        if new.phi.data_ptr() != addr:
            pytest.skip("the allocator did not reuse the address")
        x2 = fs.next()
        x.copy_(torch.as_tensor(x2))
        A.step(p.ctx, new, x, e)
        gphi, gw, glogo, _ = p.to_host(new)
        ophi, ow, ologo, _ = O.propagate(p.ham, phis, np.ones(W), O.initial_logo(p.ham, phis), x2)
        assert cmp_rel(gw, ow) < 1e-10
        assert cmp_rel(gphi, ophi, np.abs(ophi).max()) < 1e-10
        assert phase_diff(glogo, ologo) < 1e-10
        assert cmp_rel(e.cpu().numpy(), O.local_energies(p.ham, ophi)) < 1e-10
    finally:
        p.close()
