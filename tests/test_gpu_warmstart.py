"""GPU test of the learned warm start at a reduced size (in-sample n=1500,
64 landmarks, a 2x128 network, 20000 training objects): the network is
trained by the library's own kernels on converged out-of-sample solutions
the method produced, and its starts must reach the plain start's final
stress (within 1e-4 relative) for nearly every held-out object, in far
fewer transforms than the plain start used and fewer than the
nearest-in-sample start needs."""
import dataclasses

import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


def test_warm_start_beats_plain_and_nearest_starts():
    if not gpu_available():
        pytest.skip("no GPU")
    from paper_1502_03391_amd import fjofc, warmstart
    from workloads import generators as gen
    spec = dataclasses.replace(gen.config2_spec(), n=1500, in_iters=200)
    cfg = warmstart.WarmStartConfig(landmarks=64, hidden=128, depth=2, train_objects=20000,
                                    epochs=6, batch=512, chunk=10000, oos_batch=2048)
    ctx = fjofc.Context(0)
    try:
        r = warmstart.run(ctx, cfg, eval_objects=4000, spec=spec, log=lambda *_: None)
    finally:
        ctx.close()
    ev = r["eval"]
    assert ev["warm"]["reached_frac"] >= 0.95
    assert ev["warm"]["iters_mean"] < 0.5 * ev["oos_iters_cap"]
    assert ev["warm"]["iters_mean"] < ev["nearest"]["iters_mean"]
    assert ev["warm"]["iters_p50"] < 0.4 * ev["oos_iters_cap"]
