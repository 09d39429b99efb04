"""Seeded input generators for the fast-JOFC workloads.

Latent model (used by every workload): a latent sample Z ~ N(0, I_lat),
n objects; modality k is the view Y_k = Z A_k + N(0, sigma^2) noise with
A_k a lat x lat standard-Gaussian map; the within-modality dissimilarity
Delta_k is the Euclidean distance matrix of Y_k.  These stand in for the
paper's simulated data (Section 4: Gaussian points observed under several
noisy modalities, dissimilarities = interpoint distances).

Random draws use ``numpy.random.default_rng(seed)`` in a fixed order:
Z (n x lat), then for each modality k: A_k (lat x lat), noise_k (n x lat),
then the starting configuration X0 (m n x d) when one is asked for.

Distances are summed over latent coordinates one coordinate at a time in
a fixed order, so the numpy (host) and torch (device) builders give
bit-identical FP64 values, hence identical FP32 roundings.
"""
from __future__ import annotations

import dataclasses
import math
from typing import List, Optional, Sequence

import numpy as np

__all__ = [
    "InSample", "OOSBatch", "BatchedSpec",
    "latent_views", "pairwise_dist_np", "cross_dist_np",
    "pairwise_dist_torch", "cross_dist_torch",
    "uniform_wmat", "insample", "config0", "config1_spec", "config1_views",
    "oos_objects", "config2_spec", "batched_specs", "instance_views",
    "gaussian_start",
]


# --------------------------------------------------------------------------
# random draws
# --------------------------------------------------------------------------
def latent_views(seed: int, n: int, m: int, lat: int, sigma: float,
                 d: Optional[int] = None):
    """Draw Z, the maps A_k and the noisy views Y_k (all FP64).

    Returns (views, maps, X0) where X0 is an (m n) x d N(0,1) draw made
    after the views (None when d is None).
    """
    rng = np.random.default_rng(seed)
    Z = rng.standard_normal((n, lat))
    views, maps = [], []
    for _ in range(m):
        A = rng.standard_normal((lat, lat))
        noise = rng.standard_normal((n, lat)) * sigma
        views.append(Z @ A + noise)
        maps.append(A)
    X0 = rng.standard_normal((m * n, d)) if d is not None else None
    return views, maps, X0


def matched_views(seed: int, n: int = 400, m: int = 3, anomalies: int = 0):
    """The paper's matched setting (Section 4.1): Y has n rows drawn from a
    2-D Gaussian with mean (5, 5) and identity covariance, z is the range of
    all of Y's entries, and view i is Y plus independent Uniform(-z/50, z/50)
    jitter.  With anomalies > 0, the last view is built instead from a copy of
    Y whose first `anomalies` rows are redrawn from a Gaussian with mean
    (8, 8) and covariance 2 I (the anomaly setting).  Returns the m views
    (FP64, n x 2)."""
    rng = np.random.default_rng(seed)
    Y = rng.standard_normal((n, 2)) + 5.0
    z = float(Y.max() - Y.min())
    views = []
    for i in range(m):
        base = Y
        if anomalies and i == m - 1:
            base = Y.copy()
            base[:anomalies] = 8.0 + math.sqrt(2.0) * rng.standard_normal((anomalies, 2))
        views.append(base + rng.uniform(-z / 50.0, z / 50.0, size=(n, 2)))
    return views


def oos_objects(seed: int, k: int, maps: Sequence[np.ndarray], sigma: float):
    """New objects from the same latent model: k fresh latent points, viewed
    through the in-sample maps with fresh noise.  Returns a list of k x lat
    views (one per modality)."""
    rng = np.random.default_rng(seed)
    lat = maps[0].shape[0]
    Z = rng.standard_normal((k, lat))
    out = []
    for A in maps:
        out.append(Z @ A + rng.standard_normal((k, lat)) * sigma)
    return out


def gaussian_start(seed: int, shape, scale: float = 1.0) -> np.ndarray:
    """A seeded N(0, scale^2) starting configuration (FP64)."""
    return np.random.default_rng(seed).standard_normal(shape) * scale


# --------------------------------------------------------------------------
# distances (input construction only)
# --------------------------------------------------------------------------
def pairwise_dist_np(Y: np.ndarray) -> np.ndarray:
    """FP64 Euclidean distance matrix of the rows of Y (n x lat)."""
    n, lat = Y.shape
    s = np.zeros((n, n))
    for c in range(lat):
        diff = Y[:, None, c] - Y[None, :, c]
        s += diff * diff
    return np.sqrt(s)


def cross_dist_np(Ya: np.ndarray, Yb: np.ndarray) -> np.ndarray:
    """FP64 distances between rows of Ya (k x lat) and rows of Yb (n x lat)."""
    s = np.zeros((Ya.shape[0], Yb.shape[0]))
    for c in range(Ya.shape[1]):
        diff = Ya[:, None, c] - Yb[None, :, c]
        s += diff * diff
    return np.sqrt(s)


def _torch_block_dist(torch, Ya, Yb):
    s = torch.zeros((Ya.shape[0], Yb.shape[0]), dtype=torch.float64,
                    device=Ya.device)
    for c in range(Ya.shape[1]):
        diff = Ya[:, None, c] - Yb[None, :, c]
        s += diff * diff
    return torch.sqrt(s)


def pairwise_dist_torch(Y: np.ndarray, device, out=None, block: int = 512):
    """Same values as pairwise_dist_np, built on `device` in row blocks and
    stored as FP32 (n x n).  `out` may be a preallocated FP32 tensor."""
    import torch
    Yt = torch.from_numpy(np.ascontiguousarray(Y)).to(device)
    n = Y.shape[0]
    if out is None:
        out = torch.empty((n, n), dtype=torch.float32, device=device)
    for r0 in range(0, n, block):
        r1 = min(n, r0 + block)
        out[r0:r1] = _torch_block_dist(torch, Yt[r0:r1], Yt).to(torch.float32)
    return out


def cross_dist_torch(Ya: np.ndarray, Yb: np.ndarray, device, out=None,
                     block: int = 512):
    """Same values as cross_dist_np, on `device`, FP32 (k x n)."""
    import torch
    A = torch.from_numpy(np.ascontiguousarray(Ya)).to(device)
    B = torch.from_numpy(np.ascontiguousarray(Yb)).to(device)
    k = Ya.shape[0]
    if out is None:
        out = torch.empty((k, Yb.shape[0]), dtype=torch.float32, device=device)
    for r0 in range(0, k, block):
        r1 = min(k, r0 + block)
        out[r0:r1] = _torch_block_dist(torch, A[r0:r1], B).to(torch.float32)
    return out


# --------------------------------------------------------------------------
# weights
# --------------------------------------------------------------------------
def uniform_wmat(m: int, w: float, fid: float = 1.0) -> np.ndarray:
    """m x m weights of the uniform JOFC case: fidelity `fid` on the
    diagonal, commensurability `w` off it."""
    W = np.full((m, m), float(w))
    np.fill_diagonal(W, float(fid))
    return W


# --------------------------------------------------------------------------
# named workloads
# --------------------------------------------------------------------------
@dataclasses.dataclass
class InSample:
    """One in-sample problem.  delta: list of m FP32 n x n arrays (exactly
    symmetric, zero diagonal); X0: FP32 (m n) x d; wmat: FP64 m x m."""
    name: str
    m: int
    n: int
    d: int
    delta: List[np.ndarray]
    X0: np.ndarray
    wmat: np.ndarray
    iters: int
    tol: float
    stress_every: int
    views: Optional[List[np.ndarray]] = None
    maps: Optional[List[np.ndarray]] = None


def insample(name, seed, n, m, d, lat, sigma, w, iters, tol=0.0,
             stress_every=1, keep_views=False) -> InSample:
    views, maps, X0 = latent_views(seed, n, m, lat, sigma, d)
    delta = [pairwise_dist_np(Y).astype(np.float32) for Y in views]
    return InSample(name, m, n, d, delta, X0.astype(np.float32),
                    uniform_wmat(m, w), iters, tol, stress_every,
                    views if keep_views else None,
                    maps if keep_views else None)


def config0() -> InSample:
    """Plain in-sample fJOFC: m=2, n=200, d=2, 3 latent dims, noise 0.1,
    fidelity weight 1, commensurability 0.5, X0 ~ N(0,1), 200 iterations or
    relative stress change below 1e-10 (stress every iteration)."""
    return insample("insample_m2_n200_d2", 0, 200, 2, 2, 3, 0.1, 0.5,
                    200, 1e-10, 1)


@dataclasses.dataclass
class Config1Spec:
    name: str = "insample_m3_n20000_d5"
    seed: int = 1
    m: int = 3
    n: int = 20000
    d: int = 5
    lat: int = 8
    sigma: float = 0.2
    w: float = 0.5
    iters: int = 300
    stress_every: int = 10


def config1_spec() -> Config1Spec:
    """In-sample at scale: m=3, n=20000, d=5, 8 latent dims, noise 0.2,
    FP32 dissimilarities (4.8 GB), 300 iterations, stress every 10."""
    return Config1Spec()


def config1_views(spec: Optional[Config1Spec] = None):
    spec = spec or Config1Spec()
    return latent_views(spec.seed, spec.n, spec.m, spec.lat, spec.sigma, spec.d)


@dataclasses.dataclass
class OOSBatch:
    name: str
    m: int
    n: int
    d: int
    k: int


@dataclasses.dataclass
class Config2Spec:
    name: str = "oos_m2_n10000_d5_k50000"
    seed_in: int = 2
    seed_new: int = 20
    seed_train: int = 21
    seed_landmarks: int = 22
    seed_start: int = 23
    m: int = 2
    n: int = 10000
    d: int = 5
    lat: int = 8
    sigma: float = 0.2
    w: float = 0.5
    in_iters: int = 300
    k: int = 50000
    iters: int = 100
    batch: int = 4096


def config2_spec() -> Config2Spec:
    """Out-of-sample: in-sample m=2, n=10000, d=5 (300 iterations) then
    50000 new objects from the same latent model, 100 iterations each,
    4096 objects per launch."""
    return Config2Spec()


@dataclasses.dataclass
class BatchedSpec:
    idx: int
    m: int
    n: int
    d: int
    sigma: float
    seed: int


def batched_specs(count: int = 512, seed: int = 3, n_lo: int = 64,
                  n_hi: int = 2048) -> List[BatchedSpec]:
    """Uneven batch: m ~ U{2,3,4}, n ~ U[n_lo, n_hi], d ~ U{2,3,5},
    sigma ~ U[0.05, 0.3]; instance i draws its data with seed 3000 + i."""
    rng = np.random.default_rng(seed)
    ms = rng.integers(2, 5, size=count)
    ns = rng.integers(n_lo, n_hi + 1, size=count)
    ds = rng.choice(np.array([2, 3, 5]), size=count)
    sig = rng.uniform(0.05, 0.3, size=count)
    return [BatchedSpec(i, int(ms[i]), int(ns[i]), int(ds[i]), float(sig[i]),
                        3000 + i) for i in range(count)]


def instance_views(spec: BatchedSpec, lat: int = 3):
    """Views and X0 of one batched instance (latent model of the small
    in-sample workload: 3 latent dims)."""
    return latent_views(spec.seed, spec.n, spec.m, lat, spec.sigma, spec.d)
