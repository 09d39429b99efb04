"""GPU tests of the batched in-sample path (fjofc_batch_*): uneven problems
advanced in lockstep and replayed from a captured HIP graph.

Each problem in a batch runs the same kernels with the same tile shapes as
a standalone fjofc_embed, so results must be bitwise equal to it; both are
checked against the FP64 oracle at the in-sample tolerances (stress 1e-5
relative, X 1e-4 relative Frobenius).
"""
import numpy as np
import pytest

from tests.conftest import gpu_available
from workloads import generators as gen

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1502_03391_amd import fjofc
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


def _instances(count, seed=3, n_lo=16, n_hi=700):
    specs = gen.batched_specs(count, seed=seed, n_lo=n_lo, n_hi=n_hi)
    out = []
    for sp in specs:
        views, _, X0 = gen.instance_views(sp)
        delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
        out.append((sp, delta, gen.uniform_wmat(sp.m, 0.5), X0.astype(np.float32)))
    return out


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("tile", [None, "64:4", "96:5"])
def test_batch_equals_standalone_and_oracle(ctx, monkeypatch, tile):
    """Also with every instance forced onto a multi-wavefront tile variant,
    whose launches size their LDS for the tallest tile of the batch."""
    if tile:
        monkeypatch.setenv("FJOFC_TILE", tile)
    insts = _instances(12)
    iters = 40
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    b = fjofc.Batch(ctx, dev)
    res = b.run(iters, stress_every=iters)
    torch.cuda.synchronize()
    for (sp, dl, w, X0), (dd, _, Xb), r in zip(insts, dev, res):
        Xs = _dev(X0)
        rs, _ = fjofc.fjofc_embed(ctx, dd, w, Xs, iters, stress_every=iters)
        assert torch.equal(Xb, Xs), f"instance {sp.idx} differs from standalone"
        assert r["stress"] == rs["stress"] and r["iters_run"] == iters
        Xo, ro, _ = orc.embed(dl, w, X0, iters, stress_every=iters)
        assert r["stress"] == pytest.approx(ro["stress"], rel=1e-5)
        assert _rel_fro(Xb.cpu().numpy().astype(np.float64), Xo) <= 1e-4
    b.close()


def test_graph_replays_match_eager(ctx):
    """Replay the captured graph several times, with eager work and
    synchronisations in between; every replay equals the eager result."""
    insts = _instances(7, seed=5)
    iters = 25
    X0s = [_dev(X0) for *_, X0 in insts]
    dev = [([_dev(x) for x in dl], w, X0.clone()) for (_, dl, w, _), X0 in zip(insts, X0s)]
    eager = []
    for (dd, w, _), X0 in zip(dev, X0s):
        Xe = X0.clone()
        fjofc.fjofc_embed(ctx, dd, w, Xe, iters, stress_every=5)
        eager.append(Xe)
    b = fjofc.Batch(ctx, dev)
    for rep in range(4):
        for (_, _, X), X0 in zip(dev, X0s):
            X.copy_(X0)
        res = b.run(iters, stress_every=5)
        torch.cuda.synchronize()
        for (_, _, X), Xe, r in zip(dev, eager, res):
            assert torch.equal(X, Xe), f"replay {rep} differs"
            assert r["iters_run"] == iters
        # unrelated eager work between replays
        junk = torch.randn(1 << 20, device="cuda")
        junk.mul_(2.0).sum().item()
    b.close()


def test_batch_per_instance_stop_rule(ctx):
    insts = _instances(6, seed=11, n_lo=40, n_hi=300)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    res = fjofc.fjofc_embed_batched(ctx, dev, 400, tol=1e-3, tol_mode=1, stress_every=1)
    torch.cuda.synchronize()
    for (sp, dl, w, X0), r in zip(insts, res):
        _, ro, ho = orc.embed(dl, w, X0, 400, tol=1e-3, tol_mode=1, stress_every=1)
        t = ro["iters_run"]
        margin = abs((ho[t - 1] - ho[t]) - 1e-3 * ho[t - 1]) / ho[t - 1] if 0 < t < 400 else 1.0
        if margin > 1e-5:
            assert r["iters_run"] == t and r["converged"] == ro["converged"]


def test_batch_stop_rule_between_stress_checks(ctx):
    """Stop rules tested every third transform.  The transforms in between
    run each group's finalize on the group's own graph branch, and an
    instance that has stopped must be left alone there.  Every instance
    stops at the same transform, with bitwise the same X and stress, as a
    standalone run (which has a single group and no branches).  With these
    draws two of the eight instances stop early (the oracle stops them
    after 90 and 174 transforms)."""
    insts = _instances(8, seed=17, n_lo=40, n_hi=600)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    iters = 300
    b = fjofc.Batch(ctx, dev)
    res = b.run(iters, tol=1e-4, tol_mode=1, stress_every=3)
    torch.cuda.synchronize()
    stopped = 0
    for (sp, dl, w, X0), (dd, _, Xb), r in zip(insts, dev, res):
        Xs = _dev(X0)
        rs, _ = fjofc.fjofc_embed(ctx, dd, w, Xs, iters, tol=1e-4, tol_mode=1, stress_every=3)
        assert r["iters_run"] == rs["iters_run"] and r["converged"] == rs["converged"]
        assert r["stress"] == rs["stress"]
        assert torch.equal(Xb, Xs), f"instance {sp.idx} differs from standalone"
        stopped += r["iters_run"] < iters
    assert stopped >= 1
    b.close()


def test_batch_rejects_bad_problem(ctx):
    insts = _instances(3, seed=2)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    bad = dev[1][1].copy()
    bad[0, 0] = -1.0
    dev[1] = (dev[1][0], bad, dev[1][2])
    with pytest.raises(fjofc.FjofcError) as e:
        fjofc.Batch(ctx, dev)
    assert "problem 1" in str(e.value)
