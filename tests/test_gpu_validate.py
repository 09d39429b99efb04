"""GPU tests of the dissimilarity check (fjofc_validate_delta and the
FJOFC_VALIDATE hook): every rule of Section 1's Delta in R_+^{n x n}
(finite, non-negative, symmetric, zero diagonal), the first offending entry
in row-major order against the oracle's entry-by-entry scan, and the hook
in the in-sample, batched and out-of-sample calls.  Bad values are planted
on the host; the kernels only compare them."""
import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import generators as gen

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1502_03391_amd import fjofc
    from oracle import dense as odense


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = fjofc.Context(0)
    yield c
    c.close()


def _delta(n, seed=0):
    views, _, _ = gen.latent_views(seed, n, 1, 3, 0.1)
    return gen.pairwise_dist_np(views[0]).astype(np.float32)


def _check(ctx, D):
    """(index, code) from the library, with the code read from the message."""
    try:
        return fjofc.fjofc_validate_delta(ctx, torch.from_numpy(D).cuda()), 0
    except fjofc.FjofcError as e:
        assert e.code == 1
        msg = str(e)
        for code, word in ((1, "NaN"), (2, "infinite"), (3, "negative"), (4, "symmetric"),
                           (5, "diagonal")):
            if word in msg:
                return e.where, code
        raise


@pytest.mark.parametrize("n", [1, 2, 5, 64, 65, 200, 1000])
def test_valid_matrices_pass(ctx, n):
    assert _check(ctx, _delta(n, n)) == (-1, 0)


@pytest.mark.parametrize("n", [2, 7, 64, 130, 1000])
def test_each_rule_and_first_entry(ctx, n):
    """Each kind of offence at seeded positions (both triangles, the
    diagonal, tile edges), alone and several at once: the library reports
    the oracle's first offending entry and its rule."""
    rng = np.random.default_rng(n)
    base = _delta(n, 3 * n)
    for trial in range(12):
        D = base.copy()
        for _ in range(1 + trial % 3):
            i, j = (int(x) for x in rng.integers(0, n, 2))
            kind = int(rng.integers(1, 6))
            if kind == 1:
                D[i, j] = D[j, i] = np.nan
            elif kind == 2:
                D[i, j] = D[j, i] = np.inf
            elif kind == 3:
                D[i, j] = D[j, i] = -abs(D[i, j]) - 1.0
            elif kind == 4 and i != j:
                D[i, j] = D[i, j] + 0.5       # only one triangle changes
            elif kind == 5:
                D[i, i] = 0.25
        assert _check(ctx, D) == odense.first_invalid(D)


def test_hook_in_embed_batch_and_oos(ctx, monkeypatch):
    """With FJOFC_VALIDATE the computing calls reject a bad input before
    any other work (and leave X untouched); without it they do not look."""
    n, m, d = 100, 2, 2
    views, maps, X0 = gen.latent_views(4, n, m, 3, 0.1, d)
    delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
    delta[1][10, 20] += 1.0
    wmat = gen.uniform_wmat(m, 0.5)
    dd = [torch.from_numpy(x).cuda() for x in delta]
    X = torch.from_numpy(X0.astype(np.float32)).cuda()
    fjofc.fjofc_embed(ctx, dd, wmat, X.clone(), 2)          # no check without the switch
    monkeypatch.setenv("FJOFC_VALIDATE", "1")
    Xc = X.clone()
    with pytest.raises(fjofc.FjofcError) as e:
        fjofc.fjofc_embed(ctx, dd, wmat, Xc, 2)
    assert e.value.code == 1 and "Delta_1" in str(e.value) and "(10, 20)" in str(e.value)
    assert torch.equal(Xc, X)
    with pytest.raises(fjofc.FjofcError):
        fjofc.Batch(ctx, [(dd, wmat, X.clone())])
    # out of sample: delta_new must be finite and non-negative
    new = gen.oos_objects(5, 3, maps, 0.1)
    dnew = np.stack([gen.cross_dist_np(new[i], views[i]) for i in range(m)],
                    axis=1).astype(np.float32)
    Y = torch.zeros((3, m, d), device="cuda")
    fjofc.fjofc_oos(ctx, X, wmat, torch.from_numpy(dnew).cuda(), Y, 2)
    dnew[2, 1, 7] = -1.0
    with pytest.raises(fjofc.FjofcError) as e:
        fjofc.fjofc_oos(ctx, X, wmat, torch.from_numpy(dnew).cuda(), Y, 2)
    assert "object 2, modality 1, entry 7" in str(e.value)
    monkeypatch.setenv("FJOFC_VALIDATE", "0")
    fjofc.fjofc_embed(ctx, dd, wmat, X.clone(), 2)
