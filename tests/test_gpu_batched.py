"""GPU tests of the batched in-sample path (fjofc_batch_*): uneven problems
advanced together, in lockstep launches or in one persistent launch, and
replayed from a captured HIP graph.

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


LAUNCHES = ["lockstep", "persistent"]


@pytest.mark.parametrize("launch", LAUNCHES)
@pytest.mark.parametrize("tile", [None, "64:4", "96:5", "128:1", "128:0"])
def test_batch_equals_standalone_and_oracle(ctx, monkeypatch, tile, launch):
    """Also with every instance forced onto a multi-wavefront tile variant,
    whose launches size their LDS for the tallest tile of the batch, or onto
    a one-wavefront variant, single- or double-buffered (the persistent
    launch has no double-buffered form and refuses that plan)."""
    if tile:
        monkeypatch.setenv("FJOFC_TILE", tile)
    insts = _instances(12)
    iters = 40
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    if launch == "persistent" and tile == "128:0":
        with pytest.raises(fjofc.FjofcError) as e:
            fjofc.Batch(ctx, dev, launch=launch)
        assert e.value.code == 1
        return
    b = fjofc.Batch(ctx, dev, launch=launch)
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


@pytest.mark.parametrize("launch", LAUNCHES)
def test_graph_replays_match_eager(ctx, launch):
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
    b = fjofc.Batch(ctx, dev, launch=launch)
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


@pytest.mark.parametrize("seed,tol,every", [(12, 0.05, 5), (14, 0.03, 2)])
def test_batch_per_instance_stop_rule(ctx, seed, tol, every):
    """Every instance stops at the oracle's transform, with the oracle's X,
    and bitwise as its standalone run.  The draws are chosen so that every
    checkpoint decision of every instance is at least 1e-4 (relative to the
    previous stress) from the threshold; that is asserted first."""
    insts = _instances(6, seed=seed, n_lo=40, n_hi=300)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    res = fjofc.fjofc_embed_batched(ctx, dev, 400, tol=tol, tol_mode=1, stress_every=every)
    torch.cuda.synchronize()
    for (sp, dl, w, X0), (dd, _, Xb), r in zip(insts, dev, res):
        Xo, ro, ho = orc.embed(dl, w, X0, 400, tol=tol, tol_mode=1, stress_every=every)
        t = ro["iters_run"]
        assert ro["converged"] == 1 and 0 < t < 400
        for c in range(every, t + 1, every):
            prev = ho[c - every]
            assert abs((prev - ho[c]) - tol * prev) / prev >= 1e-4
        assert r["iters_run"] == t and r["converged"] == 1
        assert _rel_fro(Xb.cpu().numpy().astype(np.float64), Xo) <= 1e-4
        Xs = _dev(X0)
        rs, _ = fjofc.fjofc_embed(ctx, dd, w, Xs, 400, tol=tol, tol_mode=1, stress_every=every)
        assert torch.equal(Xb, Xs) and r["stress"] == rs["stress"]


@pytest.mark.parametrize("launch", LAUNCHES)
def test_batch_stop_rule_between_stress_checks(ctx, launch):
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
    b = fjofc.Batch(ctx, dev, launch=launch)
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


def test_persistent_and_lockstep_batches_agree(ctx):
    """The persistent launch and the lockstep graph of per-group launches
    (the default) run the same tiles and sums: bitwise equal X and results,
    with one- and four-wavefront tiles, a stop rule and stress checks every
    third transform; one plan switched between the launches (each switch
    captures again) gives the same as fresh plans."""
    insts = _instances(10, seed=21, n_lo=30, n_hi=900)
    iters = 45
    out = {}
    for mode in ("persistent", "lockstep"):
        dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
        b = fjofc.Batch(ctx, dev, launch=mode)
        res = b.run(iters, tol=2e-4, tol_mode=1, stress_every=3)
        torch.cuda.synchronize()
        out[mode] = ([X.clone() for _, _, X in dev], res)
        b.close()
    for Xp, Xl in zip(out["persistent"][0], out["lockstep"][0]):
        assert torch.equal(Xp, Xl)
    for rp, rl in zip(out["persistent"][1], out["lockstep"][1]):
        assert rp == rl
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    b = fjofc.Batch(ctx, dev)
    for mode in ("persistent", "lockstep", "persistent"):
        for (_, _, X), (*_, X0) in zip(dev, insts):
            X.copy_(_dev(X0))
        b.set_launch(mode)
        res = b.run(iters, tol=2e-4, tol_mode=1, stress_every=3)
        torch.cuda.synchronize()
        assert res == out[mode][1], mode
        for (_, _, X), Xr in zip(dev, out[mode][0]):
            assert torch.equal(X, Xr), mode
    with pytest.raises(ValueError):
        b.set_launch("other")
    assert fjofc.lib().fjofc_batch_set_launch(b._h, 7) == 1  # FJOFC_EINVAL
    b.close()


def test_persistent_batch_wider_tier(ctx):
    """Problems with d = 6..8 run in the persistent kernel's D <= 8 tier:
    bitwise equal to the lockstep graph and within tolerance of the oracle,
    beside d = 2 problems of the same batch."""
    shapes = [(2, 150, 6), (3, 97, 7), (2, 260, 8), (3, 64, 6), (2, 333, 8), (3, 120, 2)]
    insts = []
    for i, (m, n, d) in enumerate(shapes):
        sp = gen.BatchedSpec(i, m, n, d, 0.1, 5000 + i)
        views, _, X0 = gen.instance_views(sp)
        delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
        insts.append((sp, delta, gen.uniform_wmat(m, 0.5), X0.astype(np.float32)))
    iters = 30
    out = {}
    for mode in ("persistent", "lockstep"):
        dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
        b = fjofc.Batch(ctx, dev, launch=mode)
        res = b.run(iters, stress_every=iters)
        torch.cuda.synchronize()
        out[mode] = ([X.clone() for _, _, X in dev], res)
        b.close()
    for Xp, Xl in zip(out["persistent"][0], out["lockstep"][0]):
        assert torch.equal(Xp, Xl)
    assert out["persistent"][1] == out["lockstep"][1]
    for (sp, dl, w, X0), Xb, r in zip(insts, out["persistent"][0], out["persistent"][1]):
        Xo, ro, _ = orc.embed(dl, w, X0, iters, stress_every=iters)
        assert r["stress"] == pytest.approx(ro["stress"], rel=1e-5), sp.d
        assert _rel_fro(Xb.cpu().numpy().astype(np.float64), Xo) <= 1e-4, sp.d


@pytest.mark.parametrize("launch", LAUNCHES)
def test_batch_many_modalities(ctx, launch):
    """Problems with m = 6 and m = 9 beside m = 2 (the finalize's m <= 8
    and m <= 32 forms, in the branch and the persistent finalizes): every
    problem equals its standalone run bitwise and the oracle within
    tolerance."""
    shapes = [(2, 90, 3), (6, 70, 2), (9, 45, 5), (6, 111, 5), (2, 64, 2)]
    insts = []
    for i, (m, n, d) in enumerate(shapes):
        sp = gen.BatchedSpec(i, m, n, d, 0.15, 6000 + i)
        views, _, X0 = gen.instance_views(sp)
        delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
        insts.append((sp, delta, gen.uniform_wmat(m, 0.5), X0.astype(np.float32)))
    iters = 20
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    b = fjofc.Batch(ctx, dev, launch=launch)
    res = b.run(iters, stress_every=iters)
    torch.cuda.synchronize()
    for (sp, dl, w, X0), (dd, _, Xb), r in zip(insts, dev, res):
        Xs = _dev(X0)
        rs, _ = fjofc.fjofc_embed(ctx, dd, w, Xs, iters, stress_every=iters)
        assert torch.equal(Xb, Xs), f"m={sp.m} differs from standalone"
        assert r["stress"] == rs["stress"]
        Xo, ro, _ = orc.embed(dl, w, X0, iters, stress_every=iters)
        assert r["stress"] == pytest.approx(ro["stress"], rel=1e-5)
        assert _rel_fro(Xb.cpu().numpy().astype(np.float64), Xo) <= 1e-4
    b.close()


@pytest.mark.parametrize("tile", ["64:2", "64:3", "64:0"])
def test_persistent_launch_refuses_other_variants(ctx, monkeypatch, tile):
    """Tiles of 8 columns per lane (variants 2 and 3) and double-buffered
    tiles (variant 0) have no persistent form: selecting the persistent
    launch for such a batch returns FJOFC_EINVAL and leaves the plan usable
    in lockstep."""
    monkeypatch.setenv("FJOFC_TILE", tile)
    insts = _instances(3, seed=29, n_lo=30, n_hi=200)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    b = fjofc.Batch(ctx, dev)
    with pytest.raises(fjofc.FjofcError) as e:
        b.set_launch("persistent")
    assert e.value.code == 1
    res = b.run(5, stress_every=5)
    torch.cuda.synchronize()
    assert all(r["iters_run"] == 5 for r in res)
    b.close()


def test_persistent_wait_timeout_is_reported(ctx, monkeypatch):
    """A dependency wait that cannot be met (forced from the host: the first
    task waits on a counter no task increments, with a 1 ms limit) ends the
    launch early and the run returns an error instead of hanging; the same
    problems then run normally."""
    insts = _instances(4, seed=23, n_lo=30, n_hi=200)
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    monkeypatch.setenv("FJOFC_BATCH_FORCE_WAIT", "1")
    monkeypatch.setenv("FJOFC_BATCH_TIMEOUT_MS", "1")
    b = fjofc.Batch(ctx, dev, launch="persistent")
    with pytest.raises(fjofc.FjofcError) as e:
        b.run(5, stress_every=5)
    assert e.value.code == 2 and "timed out" in str(e.value)
    b.close()
    monkeypatch.delenv("FJOFC_BATCH_FORCE_WAIT")
    monkeypatch.delenv("FJOFC_BATCH_TIMEOUT_MS")
    for _, _, X in dev:
        X.zero_()
    dev = [([_dev(x) for x in dl], w, _dev(X0)) for _, dl, w, X0 in insts]
    b = fjofc.Batch(ctx, dev, launch="persistent")
    res = b.run(5, stress_every=5)
    torch.cuda.synchronize()
    for (sp, dl, w, X0), (_, _, Xb), r in zip(insts, dev, res):
        Xo, ro, _ = orc.embed(dl, w, X0, 5, stress_every=5)
        assert r["stress"] == pytest.approx(ro["stress"], rel=1e-5)
        assert _rel_fro(Xb.cpu().numpy().astype(np.float64), Xo) <= 1e-4
    b.close()

