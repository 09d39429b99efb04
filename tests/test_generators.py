"""The seeded input recipes follow the paper's description of its simulated
data (Section 4.1): checked on the draws themselves, without the GPU."""
import numpy as np

from workloads import generators as gen


def test_matched_views_recipe():
    n, m = 400, 3
    views = gen.matched_views(5, n, m)
    assert len(views) == m and all(v.shape == (n, 2) for v in views)
    # The jitter of view i is Y_i - Y; Y is not returned, but the difference
    # of two views is the difference of their jitters, each within z/50.
    mean = np.mean(views, axis=0)
    z = mean.max() - mean.min()
    for a in range(m):
        for b in range(a + 1, m):
            diff = views[a] - views[b]
            assert np.abs(diff).max() <= 2 * (z * 1.1) / 50
            # independent uniforms on (-z/50, z/50): the difference has
            # variance 2 (z/50)^2 / 3
            assert abs(diff.var() / (2 * (z / 50) ** 2 / 3) - 1) < 0.15
    # the common sample is Gaussian with mean (5, 5) and identity covariance
    assert np.allclose(mean.mean(axis=0), 5.0, atol=0.15)
    assert np.allclose(np.cov(mean.T), np.eye(2), atol=0.2)
    # seeded
    again = gen.matched_views(5, n, m)
    assert all(np.array_equal(p, q) for p, q in zip(views, again))


def test_anomaly_setting_moves_only_the_last_view():
    n, m, k = 400, 4, 10
    base = gen.matched_views(8, n, m)
    views = gen.matched_views(8, n, m, anomalies=k)
    for i in range(m - 1):
        assert np.array_equal(base[i], views[i])
    far = np.linalg.norm(views[-1] - views[0], axis=1)
    z = np.ptp(np.mean(views[:-1], axis=0))
    # rows k.. of the last view are jittered copies of Y (within 2 z/50 of
    # view 0 per coordinate); the first k are redrawn around (8, 8)
    assert far[k:].max() <= np.sqrt(2) * 2 * (z * 1.1) / 50
    assert np.mean(views[-1][:k], axis=0).min() > 6.5
    assert far[:k].mean() > 1.0
