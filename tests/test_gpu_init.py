"""GPU parity of the paper's initialisation (fjofc_init_cmds) against the
dense oracle (numpy eigh and SVD).  Eigenvectors are defined up to sign (and
the whole start up to one orthogonal transform, the orientation of the
mean's cMDS), so configurations are compared through rotation-invariant
quantities (within-block distances, the JOFC stress) and after one global
orthogonal alignment; the Ritz values are compared directly."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import generators as gen

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1502_03391_amd import fjofc
    from oracle import dense
    from oracle import structured as orc


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = fjofc.Context(0)
    yield c
    c.close()


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _gpu_init(ctx, delta, d, iters):
    m, n = len(delta), delta[0].shape[0]
    X = torch.empty((m * n, d), device="cuda")
    eig = fjofc.fjofc_init_cmds(ctx, [_dev(x) for x in delta], X, iters=iters)
    torch.cuda.synchronize()
    return X.cpu().numpy().astype(np.float64), eig


@pytest.mark.parametrize("m,n,d,lat", [(3, 400, 3, 4), (2, 257, 5, 8), (2, 120, 8, 8),
                                       (1, 64, 2, 3), (2, 6, 2, 3)])
def test_init_matches_dense_oracle(ctx, m, n, d, lat):
    views, _, _ = gen.latent_views(80 + n, n, m, lat, 0.2, d)
    delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
    Xo, eo = dense.paper_init(delta, d)
    Xg, eg = _gpu_init(ctx, delta, d, iters=80)
    np.testing.assert_allclose(eg, eo, rtol=1e-4, atol=1e-6 * np.abs(eo).max())
    for i in range(m):
        Dg = dense.distances(Xg[i * n:(i + 1) * n])
        Do = dense.distances(Xo[i * n:(i + 1) * n])
        assert np.linalg.norm(Dg - Do) <= 1e-3 * np.linalg.norm(Do)
    Q = dense.procrustes_rotation(Xg, Xo)
    assert np.linalg.norm(Xg @ Q - Xo) <= 1e-3 * np.linalg.norm(Xo)
    wmat = gen.uniform_wmat(m, 0.5)
    sg = orc.stress(delta, wmat, Xg)[0]
    so = orc.stress(delta, wmat, Xo)[0]
    assert sg == pytest.approx(so, rel=1e-3)


def test_init_of_congruent_views_has_zero_stress(ctx):
    rng = np.random.default_rng(90)
    n = 300
    Y = rng.standard_normal((n, 3)) * [3.0, 2.0, 1.0]
    views = []
    for i in range(3):
        R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
        views.append(Y @ R + rng.standard_normal(3))
    delta = [dense.distances(v).astype(np.float32) for v in views]
    Xg, _ = _gpu_init(ctx, delta, 3, iters=40)
    s = orc.stress(delta, gen.uniform_wmat(3, 0.5), Xg)[0]
    total = sum((x.astype(np.float64) ** 2).sum() / 2 for x in delta)
    assert s <= 1e-8 * total


def test_init_then_embed_beats_random_start(ctx):
    """The paper's start reaches a lower stress than the seeded random start
    after the same number of transforms (small in-sample workload)."""
    c = gen.config0()
    delta = [x.astype(np.float32) for x in c.delta]
    m, n, d = len(delta), delta[0].shape[0], c.d
    Xi, _ = _gpu_init(ctx, delta, d, iters=40)
    dd = [_dev(x) for x in delta]
    Xa = _dev(Xi)
    ra, _ = fjofc.fjofc_embed(ctx, dd, c.wmat, Xa, 50)
    Xb = _dev(c.X0)
    rb, _ = fjofc.fjofc_embed(ctx, dd, c.wmat, Xb, 50)
    assert ra["stress"] < rb["stress"]


def test_init_rejects_bad_arguments(ctx):
    views, _, _ = gen.latent_views(5, 50, 2, 3, 0.2, 2)
    dd = [_dev(gen.pairwise_dist_np(Y)) for Y in views]
    with pytest.raises(fjofc.FjofcError):
        fjofc.fjofc_init_cmds(ctx, dd, torch.empty((100, 9), device="cuda"))
    with pytest.raises(fjofc.FjofcError):
        fjofc.fjofc_init_cmds(ctx, dd, torch.empty((100, 2), device="cuda"), iters=0)
