"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: the
paper's printed closed forms (tests/golden), LAPACK/numpy pseudo-inverses,
scikit-learn's textbook SMACOF, exact identities, invariances, and
fixed points.  None of these touches the GPU.
"""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import dense, structured as orc
from oracle import dense as odense
from workloads import generators as gen

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _read_golden(name):
    rows = []
    with open(os.path.join(GOLD, name)) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            head, mat = line.split("|")
            M = np.array([[float(Fraction(x)) for x in r.split(",")]
                          for r in mat.strip().split(";")])
            rows.append((head.split(), M))
    return rows


def _problem(seed, m, n, d, lat=3, sigma=0.2, w=0.5, wmat=None):
    views, maps, X0 = gen.latent_views(seed, n, m, lat, sigma, d)
    delta = [gen.pairwise_dist_np(Y).astype(np.float32) for Y in views]
    if wmat is None:
        wmat = gen.uniform_wmat(m, w)
    return delta, wmat, X0


def _general_wmat(m, seed=5):
    rng = np.random.default_rng(seed)
    W = rng.uniform(0.2, 2.0, size=(m, m))
    W = 0.5 * (W + W.T)
    np.fill_diagonal(W, rng.uniform(0.5, 2.0, size=m))
    return W


# ---------------------------------------------------------------- closed forms
def test_winv_uniform_matches_eq_w1inv():
    """eq:W1inv (golden) vs the oracle's Gauss-Jordan inverse of eq:modW."""
    for head, M in _read_golden("winv_uniform.txt"):
        m, n, w = int(head[0]), int(head[1]), float(Fraction(head[2]))
        Wi = orc.inverse(orc.wmod(gen.uniform_wmat(m, w), n))
        np.testing.assert_allclose(Wi, M, rtol=1e-13, atol=0)


def test_winv_w3_matches_section_211():
    """eq:W3 weights: the printed closed form of W^-1 (golden)."""
    for head, M in _read_golden("winv_w3.txt"):
        n = int(head[0])
        ws = np.array([float(Fraction(x)) for x in head[1].split(",")])
        wmat = np.outer(ws, ws)
        np.fill_diagonal(wmat, ws)
        Wi = orc.inverse(orc.wmod(wmat, n))
        np.testing.assert_allclose(Wi, M, rtol=1e-13, atol=0)


def test_winv_c_scaled_form():
    """Section 2.1.1: W = c n diag(w) + diag(w)((sum w) I - J diag(w)) has
    inverse diag(w)^-1/(cn + sum w) + J/(cn (cn + sum w))."""
    ws = np.array([1.5, 0.7, 2.0])
    n, c = 9, 3.0
    m = len(ws)
    D = np.diag(ws)
    W = c * n * D + D @ (ws.sum() * np.eye(m) - np.ones((m, m)) @ D)
    closed = np.diag(1 / ws) / (c * n + ws.sum()) + np.ones((m, m)) / (c * n * (c * n + ws.sum()))
    np.testing.assert_allclose(orc.inverse(W), closed, rtol=1e-13)


def test_wmod_is_laplacian_identity_part():
    """Appendix A: L = W (x) I_n - diag(w_ii) (x) J_n with W from eq:modW."""
    m, n = 3, 5
    wmat = _general_wmat(m)
    L = dense.laplacian(dense.omnibus_weights(wmat, n))
    Wm = orc.wmod(wmat, n)
    rhs = np.kron(Wm, np.eye(n)) - np.kron(np.diag(np.diag(wmat)), np.ones((n, n)))
    np.testing.assert_allclose(L, rhs, atol=1e-13)


@pytest.mark.parametrize("m,n,w", [(2, 7, 0.5), (3, 5, 2.0), (4, 6, 10.0)])
def test_corollary1_ldagger_matches_pinv(m, n, w):
    """Corollary 1 (structured L^dagger) vs the SVD pseudo-inverse."""
    wmat = gen.uniform_wmat(m, w)
    Lp = np.linalg.pinv(dense.laplacian(dense.omnibus_weights(wmat, n)))
    np.testing.assert_allclose(dense.ldagger_corollary(wmat, n), Lp, atol=1e-12)


def test_zprime_printed_matrix():
    """The printed J_n-coefficient matrix (golden) equals its definition."""
    for head, M in _read_golden("zprime_uniform.txt"):
        m, n, w = int(head[0]), int(head[1]), float(Fraction(head[2]))
        wmat = gen.uniform_wmat(m, w)
        Wm = orc.wmod(wmat, n)
        Wi = np.linalg.inv(Wm)
        K = np.ones((m, m)) / (m * n) - np.eye(m)
        Z = -np.linalg.inv(Wm + n * K) @ K @ Wi - np.ones((m, m)) / (m * n)
        np.testing.assert_allclose(Z, M, rtol=1e-9, atol=1e-15)


def test_woodbury_kronecker_identity():
    """Remark after Theorem 1: (A(x)I + B(x)J)^-1 = A^-1(x)I - (A+nB)^-1 B A^-1 (x) J."""
    rng = np.random.default_rng(3)
    m, n = 3, 4
    A = rng.standard_normal((m, m)) + 4 * np.eye(m)
    B = rng.standard_normal((m, m))
    lhs = np.linalg.inv(np.kron(A, np.eye(n)) + np.kron(B, np.ones((n, n))))
    Ai = np.linalg.inv(A)
    rhs = np.kron(Ai, np.eye(n)) - np.kron(np.linalg.inv(A + n * B) @ B @ Ai, np.ones((n, n)))
    np.testing.assert_allclose(lhs, rhs, atol=1e-12)


def test_l22_closed_form_section3():
    """Section 3: the dense L22 block of the out-of-sample Laplacian is
    (n+mw) I - w J; its inverse is the printed L22^dagger (golden) and
    equals the inverse of eq:modW."""
    for head, M in _read_golden("l22inv_uniform.txt"):
        m, n, w = int(head[0]), int(head[1]), float(Fraction(head[2]))
        if n > 300:
            continue
        wmat = gen.uniform_wmat(m, w)
        X = np.zeros((m * n, 2))
        Wo, _, _ = dense.oos_blocks(X, wmat, np.ones((m, n)), np.zeros((m, 2)))
        L22 = dense.laplacian(Wo)[m * n:, m * n:]
        np.testing.assert_allclose(L22, (n + m * w) * np.eye(m) - w * np.ones((m, m)), atol=1e-12)
        np.testing.assert_allclose(np.linalg.inv(L22), M, rtol=1e-12)
        np.testing.assert_allclose(orc.inverse(orc.wmod(wmat, n)), M, rtol=1e-12)


# ------------------------------------------------ structured == dense (P1)
@pytest.mark.parametrize("m,n,d,kind", [
    (2, 12, 2, "uniform"), (3, 9, 3, "uniform"), (4, 8, 5, "general"),
    (3, 10, 2, "w0"), (1, 15, 3, "uniform"), (2, 11, 8, "general")])
def test_structured_step_equals_dense_pinv(m, n, d, kind):
    """eq:update with W^-1 equals pinv(L) B(X) X on the omnibus matrices."""
    wmat = {"uniform": gen.uniform_wmat(m, 0.5), "general": _general_wmat(m),
            "w0": gen.uniform_wmat(m, 0.0)}[kind]
    delta, _, X0 = _problem(11 + m * n, m, n, d)
    D = dense.omnibus_delta(delta)
    W = dense.omnibus_weights(wmat, n)
    ref = dense.guttman(X0, D, W)
    got = orc.guttman(delta, wmat, X0)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-12 * np.abs(ref).max())


def test_structured_stress_equals_dense_stress():
    m, n, d = 3, 10, 3
    wmat = _general_wmat(m)
    delta, _, X0 = _problem(4, m, n, d)
    D = dense.omnibus_delta(delta)
    W = dense.omnibus_weights(wmat, n)
    s, fid, com = orc.stress(delta, wmat, X0)
    assert s == pytest.approx(dense.stress(X0, D, W), rel=1e-13)
    assert s == pytest.approx(fid + com, rel=1e-15)


def test_b_matrix_block_diagonal():
    """Section 2.2: B(X) is block diagonal (the eta entries are 0 or NA)."""
    m, n, d = 3, 6, 2
    delta, wmat, X0 = _problem(2, m, n, d)
    B = dense.B_matrix(X0, dense.omnibus_delta(delta), dense.omnibus_weights(wmat, n))
    for i in range(m):
        for k in range(m):
            if i != k:
                assert np.all(B[i * n:(i + 1) * n, k * n:(k + 1) * n] == 0)
    for i in range(m):
        blk = B[i * n:(i + 1) * n, i * n:(i + 1) * n]
        got = orc.block_bx(delta[i], X0[i * n:(i + 1) * n], 1.0)
        np.testing.assert_allclose(got, blk @ X0[i * n:(i + 1) * n], atol=1e-12)


def test_block_bx_row_range():
    delta, wmat, X0 = _problem(8, 1, 40, 3)
    full = orc.block_bx(delta[0], X0, 1.3)
    part = orc.block_bx(delta[0], X0, 1.3, rows=(7, 23))
    np.testing.assert_array_equal(part, full[7:23])


# ----------------------------------------------------- SMACOF reductions (P2)
def _sk_smacof(D, X0, iters):
    from sklearn.manifold._mds import _smacof_single
    X, s, _ = _smacof_single(np.asarray(D, np.float64), metric=True,
                             init=X0.copy(), max_iter=iters, eps=-np.inf)
    return X, s


def test_m1_is_textbook_smacof():
    """m = 1 with unit weight: fJOFC is plain SMACOF (X+ = B(X)X / n);
    scikit-learn's implementation as the textbook reference."""
    delta, wmat, X0 = _problem(21, 1, 30, 2)
    Xo, _, _ = orc.embed(delta, gen.uniform_wmat(1, 0.0), X0, 5)
    Xs, s_sk = _sk_smacof(delta[0], X0, 5)
    np.testing.assert_allclose(Xo, Xs, atol=1e-10)
    assert orc.stress(delta, np.ones((1, 1)), Xs)[0] == pytest.approx(s_sk, rel=1e-8)


def test_w0_is_independent_smacofs():
    m, n = 3, 25
    delta, _, X0 = _problem(22, m, n, 2)
    Xo, _, _ = orc.embed(delta, gen.uniform_wmat(m, 0.0), X0, 4)
    for i in range(m):
        Xs, _ = _sk_smacof(delta[i], X0[i * n:(i + 1) * n], 4)
        np.testing.assert_allclose(Xo[i * n:(i + 1) * n], Xs, atol=1e-10)


def test_large_w_is_smacof_on_mean_delta():
    """w -> infinity forces equal blocks: SMACOF of the mean dissimilarity."""
    m, n = 2, 20
    delta, _, X0 = _problem(23, m, n, 2)
    X0 = np.vstack([X0[:n]] * m)
    Xo, _, _ = orc.embed(delta, gen.uniform_wmat(m, 1e9), X0, 3)
    mean = np.mean([d.astype(np.float64) for d in delta], axis=0)
    Xs, _ = _sk_smacof(mean, X0[:n], 3)
    for i in range(m):
        np.testing.assert_allclose(Xo[i * n:(i + 1) * n], Xs, atol=1e-6)


# ------------------------------------------------------ invariants (P3-P7)
def test_exact_euclidean_reaches_zero_stress():
    """All Delta_i = D(Y) with Y in R^d: the global minimum is sigma = 0."""
    m, n, d = 2, 30, 2
    Y = gen.gaussian_start(31, (n, d))
    D = gen.pairwise_dist_np(Y).astype(np.float32)
    X0 = np.vstack([Y, Y]) + 0.05 * gen.gaussian_start(32, (m * n, d))
    X, res, _ = orc.embed([D, D], gen.uniform_wmat(m, 0.5), X0, 300)
    # residual floor: D is FP32-rounded, so sigma cannot reach 0 exactly
    assert res["stress_norm"] < 1e-10


def test_stress_monotone_non_increasing():
    """Majorisation (eq:major): sigma never increases along the iterates."""
    delta, wmat, X0 = _problem(41, 3, 30, 2)
    _, _, hist = orc.embed(delta, wmat, X0, 100)
    assert np.all(np.diff(hist) <= 1e-12 * hist[:-1])


def test_stress_identity_eq_major():
    """sigma = sum W Delta^2 + tr X'LX - 2 tr X'B(X)X; fidelity is half the
    full-square Frobenius norm (Remark faststress); eq:comm."""
    m, n, d = 3, 12, 3
    delta, wmat, X0 = _problem(42, m, n, d)
    D = dense.omnibus_delta(delta)
    W = dense.omnibus_weights(wmat, n)
    L = dense.laplacian(W)
    B = dense.B_matrix(X0, D, W)
    iu = np.triu_indices(m * n, 1)
    ident = (W[iu] * D[iu] ** 2).sum() + np.trace(X0.T @ L @ X0) - 2 * np.trace(X0.T @ B @ X0)
    s, fid, com = orc.stress(delta, wmat, X0)
    assert s == pytest.approx(ident, rel=1e-12)
    half = 0.0
    for i in range(m):
        Xi = X0[i * n:(i + 1) * n]
        half += 0.5 * ((delta[i].astype(np.float64) - dense.distances(Xi)) ** 2).sum()
    assert fid == pytest.approx(half, rel=1e-12)
    blocks = [X0[i * n:(i + 1) * n] for i in range(m)]
    Xbar = sum(blocks) / m
    procrustes = m * sum(((b - Xbar) ** 2).sum() for b in blocks)
    assert com == pytest.approx(0.5 * procrustes, rel=1e-12)


def test_blocks_centred_after_one_step():
    """1^T B_i = 0: every block of X_t is centred whatever X_{t-1} is."""
    m, n, d = 3, 15, 3
    delta, wmat, X0 = _problem(43, m, n, d)
    X1 = orc.guttman(delta, wmat, X0 + 5.0)
    for i in range(m):
        assert np.abs(X1[i * n:(i + 1) * n].sum(0)).max() < 1e-12


def test_rotation_translation_scale_equivariance():
    m, n, d = 2, 14, 3
    delta, wmat, X0 = _problem(44, m, n, d)
    Q, _ = np.linalg.qr(np.random.default_rng(1).standard_normal((d, d)))
    b = np.array([3.0, -1.0, 2.0])
    X1 = orc.guttman(delta, wmat, X0)
    np.testing.assert_allclose(orc.guttman(delta, wmat, X0 @ Q + b), X1 @ Q, atol=1e-11)
    s = 4.0  # a power of two: scaling the FP32 dissimilarities stays exact
    sdelta = [np.float32(s) * x for x in delta]
    np.testing.assert_allclose(orc.guttman(sdelta, wmat, s * X0), s * X1, atol=1e-10)
    assert orc.stress(sdelta, wmat, s * X0)[0] == pytest.approx(s * s * orc.stress(delta, wmat, X0)[0], rel=1e-12)


def test_coincident_points_contribute_zero():
    """eq:B: d_jl = 0 gives b_jl = 0 (and stress still counts Delta^2)."""
    n, d = 6, 2
    X = gen.gaussian_start(5, (n, d))
    X[3] = X[1]
    D = gen.pairwise_dist_np(gen.gaussian_start(6, (n, 3))).astype(np.float32)
    got = orc.block_bx(D, X, 1.0)
    W = dense.omnibus_weights(np.ones((1, 1)), n)
    ref = dense.B_matrix(X, D.astype(np.float64), W) @ X
    np.testing.assert_allclose(got, ref, atol=1e-13)
    assert np.all(np.isfinite(got))


# ---------------------------------------------------------- stop rule (R2/R3)
def test_stop_rule_relative():
    delta, wmat, X0 = _problem(45, 2, 20, 2)
    _, res_full, hist = orc.embed(delta, wmat, X0, 400)
    tol = 1e-4
    X, res, h2 = orc.embed(delta, wmat, X0, 400, tol=tol, tol_mode=1)
    t = res["iters_run"]
    assert res["converged"] == 1 and 0 < t < 400
    assert hist[t - 1] - hist[t] < tol * hist[t - 1]
    # every earlier checkpoint decreased by at least the threshold
    assert np.all(hist[0:t - 1] - hist[1:t] >= tol * hist[0:t - 1])
    assert res["stress"] == pytest.approx(hist[t], rel=1e-12)


def test_stop_rule_paper_normalised_and_every():
    delta, wmat, X0 = _problem(46, 2, 20, 2)
    m, n = 2, 20
    pairs = m * n * (m * n - 1) / 2
    _, _, hist = orc.embed(delta, wmat, X0, 300)
    X, res, h = orc.embed(delta, wmat, X0, 300, tol=1e-6, tol_mode=2, stress_every=5)
    t = res["iters_run"]
    assert t % 5 == 0
    assert hist[t - 5] - hist[t] < 1e-6 * pairs
    assert np.isnan(h[t - 1]) or t - 1 == 0


def test_zero_iterations_returns_start_and_its_stress():
    delta, wmat, X0 = _problem(47, 2, 10, 2)
    X, res, _ = orc.embed(delta, wmat, X0, 0)
    np.testing.assert_array_equal(X, X0)
    assert res["stress"] == pytest.approx(orc.stress(delta, wmat, X0)[0], rel=1e-15)


# -------------------------------------------------------- out-of-sample (P8-P12)
@pytest.mark.parametrize("m,n,d,kind", [(2, 10, 2, "uniform"), (3, 8, 3, "general"),
                                        (1, 12, 2, "uniform")])
def test_oos_closed_form_equals_dense(m, n, d, kind):
    """The xi/psi update after eq:joosupdate equals the dense
    L22^-1[(B12' - L12')X + B22 y] assembled from W^(o) and B(X^(o))."""
    wmat = gen.uniform_wmat(m, 0.5) if kind == "uniform" else _general_wmat(m)
    X = gen.gaussian_start(51, (m * n, d))
    dnew = np.abs(gen.gaussian_start(52, (m, n))).astype(np.float32) + 0.5
    y = gen.gaussian_start(53, (m, d))
    ref, L22, B22 = dense.oos_step(X, wmat, dnew, y)
    np.testing.assert_allclose(orc.oos_step(X, wmat, dnew, y), ref, atol=1e-12)
    assert np.count_nonzero(B22 - np.diag(np.diag(B22))) == 0
    np.testing.assert_allclose(L22, orc.wmod(wmat, n), atol=1e-12)
    assert orc.oos_stress(X, wmat, dnew, y) == pytest.approx(dense.oos_stress(X, wmat, dnew, y), rel=1e-12)


def test_oos_m1_w0_is_single_point_smacof():
    """m = 1: the textbook single-point out-of-sample SMACOF update
    y+ = (1/n) sum_j [x_j + delta_j (y - x_j)/||y - x_j||]."""
    n, d = 20, 3
    X = gen.gaussian_start(54, (n, d))
    dn = (np.abs(gen.gaussian_start(55, (1, n))) + 0.3).astype(np.float32)
    y = gen.gaussian_start(56, (1, d))
    diff = y[0] - X
    dist = np.sqrt((diff ** 2).sum(1))
    ref = (X + dn[0].astype(np.float64)[:, None] * diff / dist[:, None]).mean(0)
    np.testing.assert_allclose(orc.oos_step(X, np.ones((1, 1)), dn, y)[0], ref, atol=1e-13)


def test_oos_leave_one_out_fixed_point():
    """At a converged in-sample X*, embedding object j out of sample against
    the other n-1 objects returns X*_j (its stress gradient vanishes)."""
    m, n, d = 2, 16, 2
    delta, wmat, X0 = _problem(57, m, n, d, sigma=0.1)
    Xs, res, _ = orc.embed(delta, wmat, X0, 6000)
    j = n - 1
    keep = [i * n + r for i in range(m) for r in range(n) if r != j]
    Xin = Xs[keep]
    dnew = np.stack([delta[i][j, :j] for i in range(m)]).astype(np.float32)
    y = np.stack([Xs[i * n + j] for i in range(m)])
    y1 = orc.oos_step(Xin, wmat, dnew, y)
    step = np.abs(orc.guttman(delta, wmat, Xs) - Xs).max()
    assert np.abs(y1 - y).max() < 1e3 * max(step, 1e-14)


def test_oos_stress_monotone_and_stop_rules():
    m, n, d, k = 2, 30, 2, 5
    X = gen.gaussian_start(58, (m * n, d))
    dn = (np.abs(gen.gaussian_start(59, (k, m, n))) + 0.5).astype(np.float32)
    Y0 = gen.gaussian_start(60, (k, m, d))
    wmat = gen.uniform_wmat(m, 0.5)
    prev = None
    for it in range(6):
        Y, st, its = orc.oos(X, wmat, dn, Y0, it)
        assert np.all(its == it)
        if prev is not None:
            assert np.all(st <= prev * (1 + 1e-12))
        prev = st
    Yf, sf, itf = orc.oos(X, wmat, dn, Y0, 50)
    target = sf * 1.01
    Yt, st, itt = orc.oos(X, wmat, dn, Y0, 50, target=target)
    assert np.all(st <= target) and np.all(itt <= 50)
    for o in range(k):
        if itt[o] > 0:
            Yp, sp, _ = orc.oos(X, wmat, dn[o:o + 1], Y0[o:o + 1], int(itt[o]) - 1)
            assert sp[0] > target[o]


def test_nearest_start_brute_force():
    # pinned by a brute-force scan written out independently: first index of
    # the smallest value per (object, modality) row
    rng = np.random.default_rng(5)
    k, m, n, d = 4, 2, 9, 3
    X = rng.standard_normal((m * n, d))
    dnew = rng.integers(0, 3, (k, m, n)).astype(float)
    Y = dense.nearest_start(X, dnew)
    for o in range(k):
        for i in range(m):
            best, bj = None, None
            for j in range(n):
                if best is None or dnew[o, i, j] < best:
                    best, bj = dnew[o, i, j], j
            assert np.array_equal(Y[o, i], X[i * n + bj])


# ---------------------------------------------------------- relaxed updates
def _majorizer(X, Y, D, W, L):
    """eq:major's majorizing function at X for the support point Y:
    sum W Delta^2 + tr X'LX - 2 tr X'B(Y)Y (it equals sigma at X = Y)."""
    iu = np.triu_indices(X.shape[0], 1)
    BY = dense.B_matrix(Y, D, W) @ Y
    return (W[iu] * D[iu] ** 2).sum() + np.trace(X.T @ L @ X) - 2 * np.trace(X.T @ BY)


@pytest.mark.parametrize("alpha", [0.4, 1.3, 1.9])
def test_relaxed_step_lies_on_symmetric_majorizer(alpha):
    """The Conclusion's relaxed update X + alpha (Gamma(X) - X): the oracle's
    step must sit where the dense majorizer of eq:major takes the same value
    as at 2 - alpha (the quadratic is symmetric about its minimiser
    Gamma(X)), below sigma(X), and above the new stress."""
    m, n, d = 2, 14, 2
    delta, wmat, X0 = _problem(61, m, n, d)
    D = dense.omnibus_delta(delta)
    W = dense.omnibus_weights(wmat, n)
    L = dense.laplacian(W)
    X1, _, _ = orc.embed(delta, wmat, X0, 1, tol_mode=0, alpha=alpha)
    X1m, _, _ = orc.embed(delta, wmat, X0, 1, tol_mode=0, alpha=2.0 - alpha)
    ga, gb = _majorizer(X1, X0, D, W, L), _majorizer(X1m, X0, D, W, L)
    s0 = dense.stress(X0, D, W)
    assert ga == pytest.approx(gb, rel=1e-11)
    assert ga <= s0 * (1 + 1e-12)
    assert dense.stress(X1, D, W) <= ga * (1 + 1e-12)
    # the two steps straddle Gamma(X0): their mean is the plain transform
    G, _, _ = orc.embed(delta, wmat, X0, 1, tol_mode=0)
    np.testing.assert_allclose(0.5 * (X1 + X1m), G, rtol=0, atol=1e-12 * np.abs(G).max())


def test_relaxed_stress_monotone():
    delta, wmat, X0 = _problem(62, 3, 30, 2)
    _, _, hist = orc.embed(delta, wmat, X0, 100, alpha=1.9)
    assert np.all(np.diff(hist) <= 1e-12 * hist[:-1])


def test_target_mode_and_relaxed_reach_target_sooner():
    """tol_mode 3 stops at the first checkpoint whose stress is <= tol; the
    relaxed transforms reach the plain run's 200-transform stress in fewer
    transforms (the acceleration the Conclusion asks for)."""
    delta, wmat, X0 = _problem(63, 2, 60, 2, lat=3, sigma=0.1)
    _, r200, hist = orc.embed(delta, wmat, X0, 200, tol_mode=0)
    target = r200["stress"] * (1 + 1e-4)
    _, rp, hp = orc.embed(delta, wmat, X0, 400, tol=target, tol_mode=3, stress_every=1)
    first = int(np.argmax(hist <= target))
    assert rp["converged"] == 1 and rp["iters_run"] == first
    _, rr, _ = orc.embed(delta, wmat, X0, 400, tol=target, tol_mode=3, stress_every=1, alpha=1.9)
    assert rr["converged"] == 1 and rr["stress"] <= target
    assert rr["iters_run"] < 0.8 * rp["iters_run"]
    # a target above the start's stress stops before any transform
    _, r0, _ = orc.embed(delta, wmat, X0, 50, tol=hist[0] * 2, tol_mode=3)
    assert r0["iters_run"] == 0 and r0["converged"] == 1


# ------------------------------------------------- the paper's initialisation
def test_cmds_recovers_euclidean_configuration():
    """Algorithm 1 step 1 on exact Euclidean distances of n points in R^d
    gives a configuration with the same distances, and P's eigenvalues are
    those of the centred Gram Y^T Y."""
    rng = np.random.default_rng(71)
    Y = rng.standard_normal((40, 3)) * [3.0, 2.0, 1.0]
    D = dense.distances(Y)
    X, lam = dense.cmds(D, 3)
    np.testing.assert_allclose(dense.distances(X), D, rtol=0, atol=1e-10 * D.max())
    Yc = Y - Y.mean(axis=0)
    np.testing.assert_allclose(lam, np.sort(np.linalg.eigvalsh(Yc.T @ Yc))[::-1], rtol=1e-10)
    np.testing.assert_allclose(X.mean(axis=0), 0.0, atol=1e-10)


def test_procrustes_reading_recovers_rotation():
    """R13: the rotation that fits xi onto xi_0 = xi R^T is R; the printed
    U V^T (SVD of xi_0^T xi) is its transpose and does not fit."""
    rng = np.random.default_rng(72)
    xi0 = rng.standard_normal((30, 3))
    R, _ = np.linalg.qr(rng.standard_normal((3, 3)))
    xi = xi0 @ R.T
    Q = dense.procrustes_rotation(xi, xi0)
    np.testing.assert_allclose(xi @ Q, xi0, atol=1e-12)
    U, _, Vt = np.linalg.svd(xi0.T @ xi)
    assert np.linalg.norm(xi @ (U @ Vt) - xi0) > 1e-3 * np.linalg.norm(xi0)


def test_paper_init_of_congruent_views_has_zero_stress():
    """When every Delta_i is the distance matrix of one configuration
    (rotated and translated copies), all blocks of X_0 coincide and the JOFC
    stress of X_0 vanishes."""
    rng = np.random.default_rng(73)
    Y = rng.standard_normal((25, 2)) * [2.0, 1.0]
    views = []
    for i in range(3):
        R, _ = np.linalg.qr(rng.standard_normal((2, 2)))
        views.append(Y @ R + rng.standard_normal(2))
    delta = [dense.distances(v).astype(np.float32) for v in views]
    X0, eig = dense.paper_init(delta, 2)
    n = 25
    for i in range(1, 3):
        np.testing.assert_allclose(X0[i * n:(i + 1) * n], X0[:n], atol=1e-5)
    s, _, _ = orc.stress(delta, gen.uniform_wmat(3, 0.5), X0)
    total = sum((x.astype(np.float64) ** 2).sum() / 2 for x in delta)
    assert s <= 1e-9 * total
    np.testing.assert_allclose(eig[1:], np.repeat(eig[:1], 3, axis=0), rtol=1e-6)


def test_first_invalid_scan_on_hand_built_matrices():
    """The dissimilarity check of the oracle on matrices whose first bad
    entry is known by construction (Section 1: Delta in R_+^{n x n},
    symmetric, zero diagonal)."""
    base = np.array([[0, 1, 2], [1, 0, 3], [2, 3, 0]], np.float32)
    assert odense.first_invalid(base) == (-1, 0)
    # symmetric changes, so only the value rule or the diagonal rule fires
    cases = [((1, 2), np.nan, (5, 1)), ((2, 0), np.inf, (2, 2)), ((0, 2), -1.0, (2, 3)),
             ((1, 1), 0.5, (4, 5))]
    for (i, j), v, want in cases:
        D = base.copy()
        D[i, j] = v
        D[j, i] = v
        assert odense.first_invalid(D) == want
    # an asymmetric pair is reported at its upper-triangle entry, even when
    # only the lower one was changed
    D = base.copy()
    D[2, 1] = 7.0
    assert odense.first_invalid(D) == (1 * 3 + 2, 4)
    # of two offences the earlier in row-major order wins
    D = base.copy()
    D[2, 2] = 1.0
    D[0, 1] = -2.0
    assert odense.first_invalid(D) == (1, 3)
