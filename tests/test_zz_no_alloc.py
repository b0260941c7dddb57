"""afqmc_cv_train_noalloc (the training entry point that allocates nothing)
against afqmc_cv_train, through the C ABI: the same network parameters,
normalisation and per-pass losses, bit for bit, on two calls in a row (the
second with fewer samples and a smaller minibatch), and its size limits."""
import numpy as np
import pytest

import afqmc_inputs as gi
from pairs import Pair

pytestmark = pytest.mark.gpu


def samples(p, ctx, nsteps, seed):
    """Features and exact exchange of the walkers along a short trajectory."""
    A, torch = p.A, p.torch
    W, G = p.W, p.ham.nchol
    w = A.Walkers.from_numpy(gi.initial_walkers(p.trial, W, noise=0.05, seed=seed))
    A.overlap(ctx, w)
    e = torch.empty((W, 3), dtype=torch.complex128, device="cuda")
    fs = gi.FieldStream(seed, W, G)
    feats, eks = [], []
    for k in range(nsteps):
        A.step(ctx, w, torch.as_tensor(fs.next(), device="cuda"), e, reortho=(k + 1) % 5 == 0)
        f = torch.empty((W, A.CV_NFEAT), dtype=torch.float64, device="cuda")
        q = torch.empty(W, dtype=torch.complex128, device="cuda")
        A.cv_collect(ctx, w, f, q)
        feats.append(f)
        eks.append(q)
    return torch.cat(feats), torch.cat(eks)


def test_noalloc_training_equals_training():
    p = Pair(gi.SMALL.system, 64, 0.005)
    A, torch = p.A, p.torch
    try:
        feat, ek = samples(p, p.ctx, 12, seed=3)           # 768 samples
        p0, n0 = A.cv_get_params(p.ctx)
        p0, n0 = p0.clone(), n0.clone()
        for n, epochs, batch in ((feat.shape[0], 4, 256), (301, 3, 40)):
            f, q = feat[:n].contiguous(), ek[:n].contiguous()
            A.cv_set_params(p.ctx, p0, n0)
            ref_loss = A.cv_train(p.ctx, f, q, epochs, batch, 2e-3).clone()
            ref_p, ref_n = (t.clone() for t in A.cv_get_params(p.ctx))
            A.cv_set_params(p.ctx, p0, n0)
            loss = torch.full((epochs,), float("nan"), dtype=torch.float64, device="cuda")
            A.cv_train_noalloc(p.ctx, f, q, epochs, batch, 2e-3, loss)
            torch.cuda.synchronize()
            got_p, got_n = A.cv_get_params(p.ctx)
            assert got_p.cpu().numpy().tobytes() == ref_p.cpu().numpy().tobytes(), n
            assert got_n.cpu().numpy().tobytes() == ref_n.cpu().numpy().tobytes(), n
            assert loss.cpu().numpy().tobytes() == ref_loss.cpu().numpy().tobytes(), n
            assert np.all(np.isfinite(loss.cpu().numpy()))
        # without a loss buffer the parameters come out the same
        A.cv_set_params(p.ctx, p0, n0)
        A.cv_train_noalloc(p.ctx, feat[:301].contiguous(), ek[:301].contiguous(), 3, 40, 2e-3)
        torch.cuda.synchronize()
        assert A.cv_get_params(p.ctx)[0].cpu().numpy().tobytes() == ref_p.cpu().numpy().tobytes()
    finally:
        p.close()


def test_noalloc_limits():
    p = Pair(gi.SMALL.system, 10, 0.005)
    A, torch = p.A, p.torch
    try:
        n = A.CV_NOALLOC_MAX_SAMPLES + 1
        feat = torch.zeros((n, A.CV_NFEAT), dtype=torch.float64, device="cuda")
        ek = torch.zeros(n, dtype=torch.complex128, device="cuda")
        with pytest.raises(A.AfqmcError) as ei:
            A.cv_train_noalloc(p.ctx, feat, ek, 1, 64, 1e-3)
        assert ei.value.status == A.ERR_UNSUPPORTED
        with pytest.raises(A.AfqmcError) as ei:
            A.cv_train_noalloc(p.ctx, feat[:1000], ek[:1000], 1, A.CV_NOALLOC_MAX_BATCH + 1, 1e-3)
        assert ei.value.status == A.ERR_UNSUPPORTED
        with pytest.raises(A.AfqmcError) as ei:
            A.cv_train_noalloc(p.ctx, feat[:1], ek[:1], 1, 1, 1e-3)
        assert ei.value.status == A.ERR_ARG
    finally:
        p.close()
