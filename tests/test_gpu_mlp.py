"""GPU parity of the warm-start network kernels (BF16 matrix cores, FP32
accumulation) against the FP64 oracle with the same BF16 rounding points.

The two sides round to BF16 at the same places, but from FP32 vs FP64
sums, so an activation that lands near a BF16 rounding boundary can differ
by one BF16 step (2^-8 relative) in a few elements.  Outputs and gradients
are therefore compared by relative Frobenius norm at 2e-3.
"""
import numpy as np
import pytest

from tests.conftest import gpu_available

pytestmark = pytest.mark.gpu

if gpu_available():
    import torch
    from paper_1502_03391_amd import fjofc
    from oracle import mlp as omlp


@pytest.fixture(scope="module")
def ctx():
    if not gpu_available():
        pytest.skip("no GPU")
    c = fjofc.Context(0)
    yield c
    c.close()


def _rel(a, b):
    return np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300)


def _net(ctx, dims, B, seed):
    params = omlp.init_params(dims, seed)
    rng = np.random.default_rng(seed + 1)
    params = [(W, (rng.standard_normal(b.shape) * 0.1).astype(np.float32)) for W, b in params]
    net = fjofc.Mlp(ctx, dims, B)
    net.set_params([torch.from_numpy(W).cuda() for W, _ in params],
                   [torch.from_numpy(b).cuda() for _, b in params])
    x = rng.standard_normal((B, dims[0])).astype(np.float32)
    y = rng.standard_normal((B, dims[-1])).astype(np.float32)
    xb = torch.from_numpy(x).cuda().to(torch.bfloat16)
    return net, params, x, y, xb


@pytest.mark.parametrize("waves", [None, "1", "4"])
@pytest.mark.parametrize("dims,B", [([64, 48, 40, 5], 37), ([512, 512, 512, 512, 5], 1024),
                                    ([100, 70, 3], 130), ([16, 16], 1)])
def test_forward_and_gradients(ctx, monkeypatch, dims, B, waves):
    """Forward output, loss and every gradient against the FP64 oracle at
    the same BF16 rounding points, with the matrix products' workgroups
    chosen by size or forced to one or to 2 x 2 wavefronts."""
    if waves:
        monkeypatch.setenv("FJOFC_GEMM_WAVES", waves)
    net, params, x, y, xb = _net(ctx, dims, B, 7 + B)
    out = net.forward(xb)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.backward(xb, torch.from_numpy(y).cuda(), loss)
    dW, db = net.get_grads()
    torch.cuda.synchronize()
    lo, go, oo = omlp.loss_and_grads([(W.astype(np.float64), b.astype(np.float64))
                                      for W, b in params], x, y, bf16=True)
    assert _rel(out.cpu().numpy(), oo) < 2e-3
    assert abs(loss.item() - lo) <= 2e-3 * lo
    for l, (gW, gb) in enumerate(go):
        assert _rel(dW[l].cpu().numpy(), gW) < 2e-3, f"dW[{l}]"
        assert _rel(db[l].cpu().numpy(), gb) < 2e-3, f"db[{l}]"


def test_adam_step_matches_oracle(ctx):
    dims, B = [40, 32, 4], 64
    net, params, x, y, xb = _net(ctx, dims, B, 3)
    p64 = [(W.astype(np.float64), b.astype(np.float64)) for W, b in params]
    opt = omlp.Adam(p64)
    yt = torch.from_numpy(y).cuda()
    for step in range(3):
        net.backward(xb, yt)
        net.adam(1e-3)
        _, g, _ = omlp.loss_and_grads(p64, x, y, bf16=True)
        p64 = opt.step(p64, g, 1e-3)
    W, b = net.get_params()
    torch.cuda.synchronize()
    for l, (Wo, bo) in enumerate(p64):
        # parameters move by ~lr per step; compare the moves
        dWg = W[l].cpu().numpy() - params[l][0]
        dWo = Wo - params[l][0]
        assert _rel(dWg, dWo) < 2e-2, f"W[{l}]"
        assert _rel(b[l].cpu().numpy() - params[l][1], bo - params[l][1]) < 2e-2


def test_training_reduces_loss(ctx):
    dims, B = [32, 64, 64, 2], 256
    rng = np.random.default_rng(0)
    x = rng.standard_normal((B, 32)).astype(np.float32)
    y = np.stack([np.sin(x[:, 0]) + x[:, 1], x[:, 2] * x[:, 3]], 1).astype(np.float32)
    params = omlp.init_params(dims, 1)
    net = fjofc.Mlp(ctx, dims, B)
    net.set_params([torch.from_numpy(W).cuda() for W, _ in params],
                   [torch.from_numpy(b).cuda() for _, b in params])
    xb = torch.from_numpy(x).cuda().to(torch.bfloat16)
    yt = torch.from_numpy(y).cuda()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    first = None
    for _ in range(200):
        net.backward(xb, yt, loss)
        net.adam(3e-3)
        if first is None:
            first = loss.item()
    assert loss.item() < 0.2 * first


def test_features_kernel(ctx):
    k, m, n, L = 37, 2, 300, 17
    rng = np.random.default_rng(9)
    dn = rng.uniform(0, 5, (k, m, n)).astype(np.float32)
    lm = rng.choice(n, L, replace=False).astype(np.int32)
    mu = rng.standard_normal(m * L).astype(np.float32)
    isd = rng.uniform(0.5, 2, m * L).astype(np.float32)
    x = torch.empty((k, m * L), dtype=torch.bfloat16, device="cuda")
    fjofc.fjofc_mlp_features(ctx, torch.from_numpy(dn).cuda(), torch.from_numpy(lm).cuda(),
                             torch.from_numpy(mu).cuda(), torch.from_numpy(isd).cuda(), x)
    ref = ((dn[:, :, lm].reshape(k, m * L) - mu) * isd)
    np.testing.assert_array_equal(x.float().cpu().numpy(), omlp.bf16_round(ref.astype(np.float32)))


@pytest.mark.parametrize("per_modality", [False, True])
def test_predict_start_layouts(ctx, per_modality):
    m, d, B = 3, 4, 50
    dims = [24, 32, (m * d) if per_modality else d]
    net, params, x, y, xb = _net(ctx, dims, B, 11)
    out = net.forward(xb).cpu().numpy()
    Y = torch.full((B, m, d), float("nan"), device="cuda")
    net.predict_start(xb, Y)
    Yc = Y.cpu().numpy()
    want = out.reshape(B, m, d) if per_modality else np.repeat(out[:, None, :], m, axis=1)
    np.testing.assert_array_equal(Yc, want)


def test_predict_start_rejects_other_widths(ctx):
    net, _, _, _, xb = _net(ctx, [24, 32, 7], 10, 5)
    with pytest.raises(fjofc.FjofcError):
        net.predict_start(xb, torch.empty((10, 2, 5), device="cuda"))
