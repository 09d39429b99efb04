"""The allocation-free out-of-sample entry point (fjofc_oos_noalloc)
against fjofc_oos, whose kernels it shares: two calls in a row on one GPU,
the second with a smaller problem (so its scratch holds the first call's
contents), each bitwise equal to fjofc_oos on the same inputs and within
the out-of-sample parity tolerance of the oracle; sizes beyond the scratch
are rejected."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import generators as gen

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1502_03391_amd import fjofc
    from oracle import structured as orc


def _problem(seed, m, n, d, k):
    views, maps, X0 = gen.latent_views(seed, n, m, 4, 0.2, d)
    delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
    wmat = gen.uniform_wmat(m, 0.5)
    X, _, _ = orc.embed(delta, wmat, X0, 20)
    X = X.astype(np.float32)
    new = gen.oos_objects(seed + 1, k, maps, 0.2)
    dnew = np.stack([gen.cross_dist_np(new[i], views[i]) for i in range(m)],
                    axis=1).astype(np.float32)
    scale = np.sqrt((X.astype(np.float64) ** 2).mean())
    Y0 = (gen.gaussian_start(seed + 2, (k, m, d)) * scale).astype(np.float32)
    return X, wmat, dnew, Y0


def _run(fn, ctx, X, wmat, dnew, Y0, iters, tol=0.0):
    k = dnew.shape[0]
    Y = torch.from_numpy(Y0).cuda()
    st = torch.empty(k, dtype=torch.float64, device="cuda")
    it = torch.empty(k, dtype=torch.int32, device="cuda")
    fn(ctx, torch.from_numpy(X).cuda(), wmat, torch.from_numpy(dnew).cuda(), Y, iters, tol=tol,
       stress_out=st, iters_out=it)
    torch.cuda.synchronize()
    return Y.cpu().numpy(), st.cpu().numpy(), it.cpu().numpy()


def test_noalloc_matches_fjofc_oos_twice():
    if not gpu_available():
        pytest.skip("no GPU")
    ctx = fjofc.Context(0)
    try:
        for (seed, m, n, d, k, iters, tol) in [(3, 3, 2999, 5, 300, 30, 0.0),
                                               (4, 2, 257, 3, 17, 25, 1e-6)]:
            X, wmat, dnew, Y0 = _problem(seed, m, n, d, k)
            Ya, sa, ia = _run(fjofc.fjofc_oos_noalloc, ctx, X, wmat, dnew, Y0, iters, tol)
            Yb, sb, ib = _run(fjofc.fjofc_oos, ctx, X, wmat, dnew, Y0, iters, tol)
            assert np.array_equal(Ya, Yb) and np.array_equal(sa, sb) and np.array_equal(ia, ib)
            if tol == 0.0:
                Yo, so, io = orc.oos(X, wmat, dnew, Y0, iters)
                assert np.array_equal(ia, io)
                np.testing.assert_allclose(sa, so, rtol=1e-5)
                np.testing.assert_allclose(Ya, Yo, rtol=0, atol=1e-4 * np.abs(X).max())
        # beyond the scratch (4 MiB) or beyond m = 8: rejected before any work
        m, n, d = 2, 70000, 8
        Xb = torch.zeros((m * n, d), device="cuda")
        with pytest.raises(fjofc.FjofcError) as e:
            fjofc.fjofc_oos_noalloc(ctx, Xb, gen.uniform_wmat(m, 0.5),
                                    torch.zeros((1, m, n), device="cuda"),
                                    torch.zeros((1, m, d), device="cuda"), 1)
        assert e.value.code == 1 and "scratch" in str(e.value)
        with pytest.raises(fjofc.FjofcError):
            fjofc.fjofc_oos_noalloc(ctx, torch.zeros((9 * 10, 2), device="cuda"),
                                    gen.uniform_wmat(9, 0.5), torch.zeros((1, 9, 10), device="cuda"),
                                    torch.zeros((1, 9, 2), device="cuda"), 1)
    finally:
        ctx.close()
