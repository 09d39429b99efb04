"""GPU test of the learned warm start at a reduced size: the network is
trained by the library's own kernels on out-of-sample solutions the method
produced, and its starts must reach the plain start's final stress (within
1e-4 relative) in fewer transforms than the plain start needed."""
import dataclasses

import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu


def test_warm_start_beats_plain_start():
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
    assert ev["warm"]["reached_frac"] >= 0.75
    assert ev["warm"]["iters_mean"] < 0.8 * ev["oos_iters_cap"]
    assert ev["warm"]["iters_p50"] < ev["oos_iters_cap"]
