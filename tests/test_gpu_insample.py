"""GPU parity of in-sample fJOFC (fjofc_embed / fjofc_stress) against the FP64
CPU oracle, through the C ABI.

Tolerances: the GPU computes distances, reciprocals and per-tile sums in
FP32 and the combine, stress and stop rule in FP64.  After 200 transforms at
the small in-sample workload the final stress must agree to 1e-5 relative
and X to 1e-4 relative Frobenius.  Single transforms agree to ~1e-6
relative per element (FP32 rounding of sums over n terms), checked at
2e-5 of the largest entry.
"""
import os

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


def _problem(seed, m, n, d, lat=3, sigma=0.2, w=0.5, wmat=None):
    views, _, X0 = gen.latent_views(seed, n, m, lat, sigma, d)
    delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
    return delta, (wmat if wmat is not None else gen.uniform_wmat(m, w)), X0.astype(np.float32)


def _general_wmat(m, seed=5):
    rng = np.random.default_rng(seed)
    W = rng.uniform(0.2, 2.0, size=(m, m))
    W = 0.5 * (W + W.T)
    np.fill_diagonal(W, rng.uniform(0.5, 2.0, size=m))
    return W


def _gpu_embed(ctx, delta, wmat, X0, iters, **kw):
    dd = [_dev(x) for x in delta]
    X = _dev(X0)
    res, hist = fjofc.fjofc_embed(ctx, dd, wmat, X, iters, **kw)
    torch.cuda.synchronize()
    return X.cpu().numpy().astype(np.float64), res, hist


def _rel_fro(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("tile", [None, "64:4", "32:5"])
def test_config0_parity(ctx, monkeypatch, tile):
    """m=2, n=200, d=2, 200 transforms, tol 1e-10 relative, stress every
    transform: final stress to 1e-5 relative, X to 1e-4 relative Frobenius;
    with the tuned tiles and with tiles shared by several wavefronts."""
    if tile:
        monkeypatch.setenv("FJOFC_TILE", tile)
    P = gen.config0()
    Xo, ro, ho = orc.embed(P.delta, P.wmat, P.X0, P.iters, tol=P.tol, tol_mode=1,
                           stress_every=P.stress_every)
    Xg, rg, hg = _gpu_embed(ctx, P.delta, P.wmat, P.X0, P.iters, tol=P.tol,
                            tol_mode=1, stress_every=P.stress_every, want_hist=True)
    assert rg["iters_run"] == ro["iters_run"]
    assert rg["converged"] == ro["converged"]
    assert abs(rg["stress"] - ro["stress"]) <= 1e-5 * ro["stress"]
    assert _rel_fro(Xg, Xo) <= 1e-4
    ok = ~np.isnan(ho)
    assert np.array_equal(ok, ~np.isnan(hg))
    np.testing.assert_allclose(hg[ok], ho[ok], rtol=1e-5)
    # majorisation: non-increasing up to FP32 noise
    assert np.all(np.diff(hg[ok]) <= 1e-6 * hg[ok][:-1])


@pytest.mark.parametrize("tile", ["256:0", "128:1", "64:2", "512:3", "512:1", "32:1", "16:2",
                                  "24:1", "96:3", "160:0", "200:2",
                                  "512:4", "96:4", "200:4", "256:5", "48:5",
                                  "384:1", "384:4"])
@pytest.mark.parametrize("m,n,d", [(1, 2, 1), (2, 3, 2), (3, 7, 3), (2, 64, 5),
                                   (2, 255, 2), (3, 256, 5), (2, 257, 3),
                                   (4, 300, 8), (2, 513, 4), (3, 1000, 5),
                                   (2, 1030, 6), (2, 777, 7)])
def test_one_transform_parity(ctx, monkeypatch, tile, m, n, d):
    """One Guttman transform and the stress of X0 and X1, across tile shapes
    (heights that are powers of two or only multiples of 8; one wavefront or
    R x C wavefronts per tile, including heights rounded up to whole 8-row
    groups per wavefront), ragged tails (n not a multiple of the tile or of
    4) and all d.  A height above the tile width that is not a multiple of
    it gives a row padding that is not a multiple of 256 (n = 513, 777 with
    height 384), which the commensurability partials must not over-count."""
    monkeypatch.setenv("FJOFC_TILE", tile)
    wmat = _general_wmat(m, seed=n)
    delta, _, X0 = _problem(100 + n + d, m, n, d, wmat=wmat)
    X1o = orc.guttman(delta, wmat, X0)
    Xg, rg, hg = _gpu_embed(ctx, delta, wmat, X0, 1, want_hist=True)
    scale = np.abs(X1o).max()
    np.testing.assert_allclose(Xg, X1o, rtol=0, atol=2e-5 * scale)
    s0 = orc.stress(delta, wmat, X0)[0]
    s1 = orc.stress(delta, wmat, X1o)[0]
    assert hg[0] == pytest.approx(s0, rel=2e-6)
    assert rg["stress"] == pytest.approx(s1, rel=2e-5)


@pytest.mark.parametrize("m,n,d", [(2, 3600, 3), (2, 7000, 5), (2, 14000, 2), (2, 3000, 4),
                                   (2, 2500, 8), (1, 4100, 1), (2, 5000, 6), (2, 2200, 7)])
def test_one_transform_parity_table_tiles_mid_sizes(ctx, monkeypatch, m, n, d):
    """One transform at mid-size n with the tiles the tile cache picks there
    (shared 4 x 1 and 2 x 2 wavefront tiles several hundred rows tall; d = 1,
    4, 6, 7, 8 have no rows of their own and take the nearest d's), against
    the oracle."""
    monkeypatch.delenv("FJOFC_TILE", raising=False)
    th, var = fjofc.fjofc_tile_choice(ctx, n, d)
    assert th >= 8 and 0 <= var <= 5
    wmat = _general_wmat(m, seed=n)
    delta, _, X0 = _problem(500 + d, m, n, d, wmat=wmat)
    X1o = orc.guttman(delta, wmat, X0)
    Xg, rg, hg = _gpu_embed(ctx, delta, wmat, X0, 1, want_hist=True)
    np.testing.assert_allclose(Xg, X1o, rtol=0, atol=2e-5 * np.abs(X1o).max())
    assert hg[0] == pytest.approx(orc.stress(delta, wmat, X0)[0], rel=2e-6)
    assert rg["stress"] == pytest.approx(orc.stress(delta, wmat, X1o)[0], rel=2e-5)


@pytest.mark.parametrize("tile,n", [("264:1", 268), ("264:1", 530), ("392:0", 300)])
def test_tall_tiles_padding_rows(ctx, monkeypatch, tile, n):
    """A tile taller than it is wide gives a row padding that is not a
    multiple of the finalize's 256-row blocks, so the finalize never writes
    the last padding rows that boundary tiles read (masked).  They must
    hold zeros even when the workspace held NaN before: after a run of a
    larger problem from an all-NaN configuration (which leaves NaN across
    the context workspace), 3 transforms against the oracle."""
    m, d = 2, 3
    big, _, _ = _problem(299, m, 1500, d)
    Xnan = np.full((m * 1500, d), np.nan, np.float32)
    fjofc.fjofc_embed(ctx, [_dev(x) for x in big], gen.uniform_wmat(m, 0.5), _dev(Xnan), 2)
    monkeypatch.setenv("FJOFC_TILE", tile)
    wmat = _general_wmat(m, seed=n)
    delta, _, X0 = _problem(300 + n, m, n, d, wmat=wmat)
    Xo, ro, _ = orc.embed(delta, wmat, X0, 3)
    Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 3)
    assert np.all(np.isfinite(Xg))
    np.testing.assert_allclose(Xg, Xo, rtol=0, atol=2e-5 * np.abs(Xo).max())
    assert rg["stress"] == pytest.approx(ro["stress"], rel=2e-5)


def test_stress_entry_point(ctx):
    m, n, d = 3, 333, 4
    wmat = _general_wmat(m)
    delta, _, X0 = _problem(7, m, n, d, wmat=wmat)
    r = fjofc.fjofc_stress(ctx, [_dev(x) for x in delta], wmat, _dev(X0))
    s, fid, com = orc.stress(delta, wmat, X0)
    assert r["stress"] == pytest.approx(s, rel=2e-6)
    assert r["fidelity"] == pytest.approx(fid, rel=2e-6)
    assert r["commens"] == pytest.approx(com, rel=2e-6)
    assert r["iters_run"] == 0


def test_many_iterations_parity_general_w(ctx):
    m, n, d = 3, 600, 3
    wmat = _general_wmat(m, seed=9)
    delta, _, X0 = _problem(8, m, n, d, wmat=wmat)
    Xo, ro, _ = orc.embed(delta, wmat, X0, 60, stress_every=7)
    Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 60, stress_every=7)
    assert rg["iters_run"] == 60
    assert rg["stress"] == pytest.approx(ro["stress"], rel=1e-5)
    assert _rel_fro(Xg, Xo) <= 1e-4


def test_uniform_weight_entry_point(ctx):
    """fjofc_embed_w (eq:W's uniform weights) is fjofc_embed with the
    matrix w_ii = 1, w_ik = w: bitwise the same X, stress and history, and
    the oracle's result."""
    m, n, d, w = 3, 150, 2, 0.7
    delta, _, X0 = _problem(17, m, n, d)
    dd = [_dev(x) for x in delta]
    Xa, Xb = _dev(X0), _dev(X0)
    ra, ha = fjofc.fjofc_embed_w(ctx, dd, w, Xa, 25, stress_every=5, want_hist=True)
    rb, hb = fjofc.fjofc_embed(ctx, dd, gen.uniform_wmat(m, w), Xb, 25, stress_every=5,
                               want_hist=True)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb) and ra == rb and ra["iters_run"] == 25
    np.testing.assert_array_equal(ha, hb)
    Xo, ro, _ = orc.embed(delta, gen.uniform_wmat(m, w), X0, 25, stress_every=5)
    assert ra["stress"] == pytest.approx(ro["stress"], rel=1e-5)
    assert _rel_fro(Xa.cpu().numpy().astype(np.float64), Xo) <= 1e-4


@pytest.mark.parametrize("m,n,d", [(5, 70, 3), (6, 130, 2), (8, 61, 4), (9, 41, 5),
                                   (12, 33, 2)])
def test_many_modalities_parity(ctx, m, n, d):
    """m above 4 takes the finalize's wider forms (m <= 8 and m <= 32
    register tiers): X and the stress after 12 transforms with a general
    weight matrix, against the oracle."""
    wmat = _general_wmat(m, seed=m + n)
    delta, _, X0 = _problem(30 + m, m, n, d, wmat=wmat)
    Xo, ro, _ = orc.embed(delta, wmat, X0, 12, stress_every=12)
    Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 12, stress_every=12)
    assert rg["iters_run"] == 12
    assert rg["stress"] == pytest.approx(ro["stress"], rel=1e-5)
    assert _rel_fro(Xg, Xo) <= 1e-4


# (seed, tol_mode, tol, stress_every): cases whose every checkpoint decision
# lies at least 1e-4 (relative to the previous stress) away from the
# threshold in the oracle, so FP32 rounding cannot flip any of them.
STOP_CASES = [(12, 1, 5e-3, 1), (12, 1, 1e-2, 5), (43, 1, 1e-3, 1), (41, 1, 2e-3, 5),
              (12, 2, 1e-4, 1), (12, 2, 2e-4, 5), (43, 2, 1e-4, 1), (41, 2, 1e-4, 5)]


@pytest.mark.parametrize("seed,mode,tol,every", STOP_CASES)
def test_stop_rule_matches_oracle(ctx, seed, mode, tol, every):
    """Algorithm 2's stop test (relative and the paper's normalised form):
    the GPU stops at the oracle's transform and returns its X.  Every
    checkpoint's decision margin is asserted first, so the comparison is
    never skipped."""
    m, n, d = 2, 300, 2
    delta, wmat, X0 = _problem(seed, m, n, d)
    Xo, ro, ho = orc.embed(delta, wmat, X0, 500, tol=tol, tol_mode=mode, stress_every=every)
    t = ro["iters_run"]
    assert ro["converged"] == 1 and 0 < t < 500
    for c in range(every, t + 1, every):
        prev = ho[c - every]
        thr = tol * prev if mode == 1 else tol * (m * n) * (m * n - 1) / 2
        assert abs((prev - ho[c]) - thr) / prev >= 1e-4, f"checkpoint {c} within noise"
    Xg, rg, hg = _gpu_embed(ctx, delta, wmat, X0, 500, tol=tol, tol_mode=mode,
                            stress_every=every, want_hist=True)
    assert rg["iters_run"] == t and rg["converged"] == 1
    assert _rel_fro(Xg, Xo) <= 1e-4
    assert rg["stress"] == pytest.approx(ro["stress"], rel=1e-5)
    ok = ~np.isnan(ho[: t + 1])
    np.testing.assert_allclose(hg[: t + 1][ok], ho[: t + 1][ok], rtol=1e-5)


def test_early_stop_enqueues_at_most_one_chunk_past_the_stop(ctx):
    """A run capped at 5000 transforms that stops after a few: transforms
    are enqueued in chunks of 32 and the host checks the done flag of the
    chunk before the one it just enqueued, so at most two chunks of stream
    launches are issued before the stop is seen (plus the closing stress
    pass), and the result is the oracle's."""
    m, n, d = 2, 300, 2
    delta, wmat, X0 = _problem(12, m, n, d)
    tol, every = 0.2, 1
    Xo, ro, ho = orc.embed(delta, wmat, X0, 5000, tol=tol, tol_mode=1, stress_every=every)
    t = ro["iters_run"]
    assert ro["converged"] == 1 and 0 < t < 32
    for c in range(1, t + 1):
        assert abs((ho[c - 1] - ho[c]) / ho[c - 1] - tol) >= 1e-4
    fjofc.fjofc_profile_enable(ctx, True)
    try:
        Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 5000, tol=tol, tol_mode=1,
                               stress_every=every)
        prof = fjofc.fjofc_profile_read(ctx)
    finally:
        fjofc.fjofc_profile_enable(ctx, False)
    assert rg["iters_run"] == t and rg["converged"] == 1
    assert _rel_fro(Xg, Xo) <= 1e-4
    assert prof["stream_launches"] <= 2 * 32
    assert prof["edge_launches"] == 1


def test_zero_iterations_and_coincident_points(ctx):
    m, n, d = 2, 200, 3
    delta, wmat, X0 = _problem(13, m, n, d)
    X0[5] = X0[17]
    X0[n + 3] = X0[n + 100]
    Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 0)
    np.testing.assert_array_equal(Xg, X0.astype(np.float64))
    assert rg["stress"] == pytest.approx(orc.stress(delta, wmat, X0)[0], rel=2e-6)
    X1o = orc.guttman(delta, wmat, X0)
    Xg1, _, _ = _gpu_embed(ctx, delta, wmat, X0, 1)
    assert np.all(np.isfinite(Xg1))
    np.testing.assert_allclose(Xg1, X1o, rtol=0, atol=2e-5 * np.abs(X1o).max())


def test_deterministic_and_resumable(ctx):
    """Same inputs give bitwise-equal results; Algorithm 2's loop state is X
    alone, so 10 + 10 transforms equal 20."""
    m, n, d = 3, 700, 5
    delta, wmat, X0 = _problem(14, m, n, d)
    dd = [_dev(x) for x in delta]
    Xa = _dev(X0)
    fjofc.fjofc_embed(ctx, dd, wmat, Xa, 20)
    Xb = _dev(X0)
    fjofc.fjofc_embed(ctx, dd, wmat, Xb, 20)
    Xc = _dev(X0)
    fjofc.fjofc_embed(ctx, dd, wmat, Xc, 10)
    fjofc.fjofc_embed(ctx, dd, wmat, Xc, 10)
    torch.cuda.synchronize()
    assert torch.equal(Xa, Xb)
    assert torch.equal(Xa, Xc)


def test_invalid_arguments_are_rejected(ctx):
    delta, wmat, X0 = _problem(15, 2, 50, 2)
    dd = [_dev(x) for x in delta]
    bad = wmat.copy()
    bad[0, 0] = 0.0
    with pytest.raises(fjofc.FjofcError) as e:
        fjofc.fjofc_embed(ctx, dd, bad, _dev(X0), 1)
    assert e.value.code == 1
    asym = wmat.copy()
    asym[0, 1] = 0.7
    with pytest.raises(fjofc.FjofcError):
        fjofc.fjofc_embed(ctx, dd, asym, _dev(X0), 1)
    with pytest.raises(fjofc.FjofcError):
        fjofc.fjofc_embed(ctx, dd, wmat, _dev(np.zeros((100, 9))), 1)
    with pytest.raises(fjofc.FjofcError):
        fjofc.fjofc_embed(ctx, dd, wmat, _dev(X0), 1, stress_every=0)


@pytest.mark.parametrize("alpha", [0.6, 1.5, 1.9])
def test_relaxed_transforms_parity(ctx, alpha):
    """fjofc_embed_relaxed against the oracle's relaxed loop, general W and a
    ragged n; stress history non-increasing (R16's FP32 slack)."""
    m, n, d = 3, 517, 3
    wmat = _general_wmat(m, seed=21)
    delta, _, X0 = _problem(22, m, n, d, wmat=wmat)
    Xo, ro, ho = orc.embed(delta, wmat, X0, 40, stress_every=4, alpha=alpha)
    Xg, rg, hg = _gpu_embed(ctx, delta, wmat, X0, 40, stress_every=4, alpha=alpha,
                            want_hist=True)
    assert rg["iters_run"] == 40
    assert rg["stress"] == pytest.approx(ro["stress"], rel=1e-5)
    assert _rel_fro(Xg, Xo) <= 1e-4
    h = hg[~np.isnan(hg)]
    assert np.all(np.diff(h) <= 1e-6 * h[:-1])


def test_target_stop_matches_oracle(ctx):
    """FJOFC_TOL_TARGET: stop at the first checkpoint with sigma <= tol, for
    plain and relaxed transforms; at t = 0 when X0 already meets it."""
    m, n, d = 2, 300, 2
    delta, wmat, X0 = _problem(23, m, n, d)
    _, r60, hist = orc.embed(delta, wmat, X0, 60, tol_mode=0)
    target = r60["stress"] * (1 + 1e-3)
    for alpha in (1.0, 1.9):
        Xo, ro, ho = orc.embed(delta, wmat, X0, 200, tol=target, tol_mode=3, alpha=alpha)
        Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 200, tol=target, tol_mode=3, alpha=alpha)
        t = ro["iters_run"]
        assert ro["converged"] == 1 and 0 < t < 200
        # decisions within FP32 noise of the target are not compared
        if ho[t - 1] > target * (1 + 1e-5) and ho[t] < target * (1 - 1e-5):
            assert rg["iters_run"] == t and rg["converged"] == 1
            assert _rel_fro(Xg, Xo) <= 1e-4
    Xg, rg, _ = _gpu_embed(ctx, delta, wmat, X0, 50, tol=hist[0] * 2, tol_mode=3)
    assert rg["iters_run"] == 0 and rg["converged"] == 1
    np.testing.assert_array_equal(Xg, X0.astype(np.float64))


def test_relaxation_factor_is_validated(ctx):
    delta, wmat, X0 = _problem(24, 2, 40, 2)
    dd = [_dev(x) for x in delta]
    for alpha in (0.0, 2.0, -1.0, float("nan")):
        with pytest.raises(fjofc.FjofcError):
            fjofc.fjofc_embed(ctx, dd, wmat, _dev(X0), 1, alpha=alpha)
