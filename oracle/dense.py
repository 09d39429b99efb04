"""Dense numpy tier of the oracle (test infrastructure only).

This is plain JOFC as Algorithm 1 states it on the omnibus matrices, with
no structure used: the mn x mn weight matrix of eq:W2, the omnibus
dissimilarity of eq:jofcdelta (the NA entries carry weight 0), the
combinatorial Laplacian L = D - W, B(X) of eq:B, and the Moore-Penrose
pseudo-inverse from numpy (SVD).  Small mn only.
"""
from __future__ import annotations

import numpy as np


def omnibus_weights(wmat: np.ndarray, n: int) -> np.ndarray:
    """eq:W2: w_ii (J_n - I_n) on diagonal blocks, w_ij I_n off them."""
    m = wmat.shape[0]
    W = np.zeros((m * n, m * n))
    I = np.eye(n)
    J = np.ones((n, n))
    for i in range(m):
        for j in range(m):
            blk = wmat[i, i] * (J - I) if i == j else wmat[i, j] * I
            W[i * n:(i + 1) * n, j * n:(j + 1) * n] = blk
    return W


def omnibus_delta(delta) -> np.ndarray:
    """eq:jofcdelta with the eta blocks: 0 for the same object across
    modalities, NA (stored as 0, weight 0 in eq:W2) elsewhere."""
    m = len(delta)
    n = delta[0].shape[0]
    D = np.zeros((m * n, m * n))
    for i in range(m):
        D[i * n:(i + 1) * n, i * n:(i + 1) * n] = np.asarray(delta[i], np.float64)
    return D


def laplacian(W: np.ndarray) -> np.ndarray:
    return np.diag(W.sum(axis=1)) - W


def distances(X: np.ndarray) -> np.ndarray:
    diff = X[:, None, :] - X[None, :, :]
    return np.sqrt((diff * diff).sum(-1))


def B_matrix(X: np.ndarray, D: np.ndarray, W: np.ndarray) -> np.ndarray:
    """eq:B: -W_ij D_ij / d_ij off the diagonal (0 where d_ij = 0), the
    diagonal making each row sum to zero."""
    dist = distances(X)
    N = X.shape[0]
    B = np.zeros((N, N))
    off = ~np.eye(N, dtype=bool)
    nz = off & (dist != 0)
    B[nz] = -W[nz] * D[nz] / dist[nz]
    B[np.arange(N), np.arange(N)] = -B.sum(axis=1)
    return B


def stress(X: np.ndarray, D: np.ndarray, W: np.ndarray) -> float:
    """sum_{i<j} W_ij (D_ij - d_ij(X))^2 over the omnibus matrix."""
    dist = distances(X)
    iu = np.triu_indices(X.shape[0], 1)
    return float((W[iu] * (D[iu] - dist[iu]) ** 2).sum())


def guttman(X: np.ndarray, D: np.ndarray, W: np.ndarray, Lpinv=None):
    """X_t = L^dagger B(X) X with L^dagger = pinv(L)."""
    if Lpinv is None:
        Lpinv = np.linalg.pinv(laplacian(W))
    return Lpinv @ (B_matrix(X, D, W) @ X)


def ldagger_corollary(wmat: np.ndarray, n: int) -> np.ndarray:
    """Corollary 1: L^dagger = W^-1 (x) I_n + [-(W + n(J_m/mn - diag w_ii))^-1
    (J_m/mn - diag w_ii) W^-1 - J_m/mn] (x) J_n, with W the eq:modW matrix
    (formed here directly from its definition)."""
    m = wmat.shape[0]
    Wm = np.diag(n * np.diag(wmat) + (wmat.sum(1) - np.diag(wmat))) - (wmat - np.diag(np.diag(wmat)))
    Wi = np.linalg.inv(Wm)
    Jm = np.ones((m, m))
    K = Jm / (m * n) - np.diag(np.diag(wmat))
    Z = -np.linalg.inv(Wm + n * K) @ K @ Wi - Jm / (m * n)
    return np.kron(Wi, np.eye(n)) + np.kron(Z, np.ones((n, n)))


# ----------------------------------------------------------------------------
# out-of-sample, dense (Section 3): the m(n+1) omnibus with the new object's
# m copies appended after the in-sample block.
# ----------------------------------------------------------------------------
def oos_blocks(X, wmat, dnew, y):
    """Assemble W^(o), Delta^(o), X^(o) for one new object (eq:W2 weights:
    w_ii between a new copy and its own modality's in-sample points, w_ik
    between the new copies; no weight to other modalities' points)."""
    m, n = dnew.shape
    N = m * n
    Wo = np.zeros((N + m, N + m))
    Do = np.zeros((N + m, N + m))
    for i in range(m):
        rows = slice(i * n, (i + 1) * n)
        Wo[rows, N + i] = wmat[i, i]
        Wo[N + i, rows] = wmat[i, i]
        Do[rows, N + i] = dnew[i]
        Do[N + i, rows] = dnew[i]
        for k in range(m):
            if k != i:
                Wo[N + i, N + k] = wmat[i, k]
    Xo = np.vstack([X, y])
    return Wo, Do, Xo


def oos_step(X, wmat, dnew, y):
    """y_t = L22^-1 [(B12^T - L12^T) X + B22 y] (eq:joosupdate), all blocks
    taken from the dense L^(o) and B(X^(o)) (in-sample weights are zero so
    L11, B11 play no part)."""
    m, n = dnew.shape
    N = m * n
    Wo, Do, Xo = oos_blocks(X, wmat, np.asarray(dnew, np.float64), y)
    L = laplacian(Wo)
    B = B_matrix(Xo, Do, Wo)
    L12, L22 = L[:N, N:], L[N:, N:]
    B12, B22 = B[:N, N:], B[N:, N:]
    rhs = (B12.T - L12.T) @ X + B22 @ y
    return np.linalg.solve(L22, rhs), L22, B22


def oos_stress(X, wmat, dnew, y):
    """sum_{i<j} W^(o)_ij (Delta^(o)_ij - d_ij(X^(o)))^2 restricted to pairs
    that involve a new copy (the in-sample part is a constant)."""
    m, n = dnew.shape
    N = m * n
    Wo, Do, Xo = oos_blocks(X, wmat, np.asarray(dnew, np.float64), y)
    dist = distances(Xo)
    s = 0.0
    for a in range(N, N + m):
        for b in range(a):
            s += Wo[a, b] * (Do[a, b] - dist[a, b]) ** 2
    return float(s)


def nearest_start(X: np.ndarray, dnew: np.ndarray) -> np.ndarray:
    """Comparison start for the out-of-sample problem (not the paper's, which
    starts at random): for every new object o and modality i, the in-sample
    point X^(i)_j whose dissimilarity to o is smallest (numpy's argmin takes
    the first of tied minima).  X: (m n) x d, dnew: k x m x n -> k x m x d."""
    k, m, n = dnew.shape
    d = X.shape[1]
    Y = np.empty((k, m, d), dtype=X.dtype)
    for o in range(k):
        for i in range(m):
            j = int(np.argmin(dnew[o, i]))
            Y[o, i] = X[i * n + j]
    return Y


def cmds(D: np.ndarray, d: int):
    """Classical MDS (Algorithm 1 step 1): the d largest eigenpairs of
    P = -1/2 J (D o D) J, J = I - 11^T/n (numpy's eigh); returns
    X = U diag(max(lambda, 0))^(1/2) and the eigenvalues (descending)."""
    D = np.asarray(D, dtype=np.float64)
    n = D.shape[0]
    J = np.eye(n) - 1.0 / n
    P = -0.5 * J @ (D * D) @ J
    w, U = np.linalg.eigh(0.5 * (P + P.T))
    idx = np.argsort(w)[::-1][:d]
    return U[:, idx] * np.sqrt(np.maximum(w[idx], 0.0)), w[idx]


def procrustes_rotation(xi: np.ndarray, xi0: np.ndarray) -> np.ndarray:
    """Orthogonal Q minimising ||xi Q - xi0||_F: with xi^T xi0 = U S V^T,
    Q = U V^T (numpy's SVD).  Algorithm 2 prints xi_i U V^T with U S V^T the
    SVD of xi_0^T xi_i, which is the transpose of this Q."""
    U, _, Vt = np.linalg.svd(xi.T @ xi0)
    return U @ Vt


def paper_init(delta, d: int):
    """Algorithm 2's start: cMDS of the mean dissimilarity (xi_0), cMDS of
    each Delta_i centred, Procrustes fit onto xi_0; stacked modality-major.
    Returns (X0, eigenvalues (m + 1) x d)."""
    m = len(delta)
    Dm = sum(np.asarray(x, dtype=np.float64) for x in delta) / m
    xi0, e0 = cmds(Dm, d)
    xi0 = xi0 - xi0.mean(axis=0)
    blocks, eigs = [], [e0]
    for x in delta:
        xi, e = cmds(x, d)
        xi = xi - xi.mean(axis=0)
        blocks.append(xi @ procrustes_rotation(xi, xi0))
        eigs.append(e)
    return np.vstack(blocks), np.array(eigs)


# Offence codes of the dissimilarity check (Section 1: Delta in R_+^{n x n},
# symmetric with a zero diagonal).
OFFENCES = {1: "nan", 2: "inf", 3: "negative", 4: "asymmetric", 5: "diagonal"}


def first_invalid(delta: np.ndarray):
    """Scan an n x n dissimilarity entry by entry in row-major order and
    return (index i n + j, offence code) of the first entry that is NaN (1),
    infinite (2), negative (3), above the diagonal and unequal to its mirror
    entry (4), or a non-zero diagonal entry (5); (-1, 0) when none is.
    An entry's own value is judged before the diagonal and symmetry rules."""
    D = np.asarray(delta, np.float32)
    n = D.shape[0]
    for i in range(n):
        for j in range(n):
            v = D[i, j]
            if np.isnan(v):
                return i * n + j, 1
            if np.isinf(v):
                return i * n + j, 2
            if v < 0:
                return i * n + j, 3
            if i == j and v != 0:
                return i * n + j, 5
            if i < j and v != D[j, i]:
                return i * n + j, 4
    return -1, 0
