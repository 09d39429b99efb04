"""GPU parity of the warm-start network kernels (BF16 matrix cores, FP32
accumulation) against the FP64 oracle with the same BF16 rounding points.

The two sides round to BF16 at the same places, but from FP32 vs FP64
sums, so an activation or gradient that lands near a BF16 rounding boundary
can round one BF16 step apart, and that step reaches later products.
Outputs and gradients are therefore compared element by element in units
of one BF16 step (2^-7 of the element's binade, taken at least at the
array's RMS so that elements near zero are judged on the array's scale):
every element within one step, and at most 0.1% of them (and at least 2
allowed) beyond half a step.  An FP32-accumulation emulation of the GPU's
arithmetic on the host stays within 0.53 step, with 5 of 262144 elements
beyond half a step in the widest gradient.
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


def _bf16_steps(g, o):
    """|g - o| in BF16 steps of max(|o|, rms(o)) per element."""
    o = np.asarray(o, np.float64)
    g = np.asarray(g, np.float64)
    rms = np.sqrt((o * o).mean()) if o.size else 0.0
    ref = np.maximum(np.maximum(np.abs(o), rms), 1e-30)
    step = 2.0 ** (np.floor(np.log2(ref)) - 7)
    return np.abs(g - o) / step


def _assert_bf16_close(g, o, what):
    s = _bf16_steps(g, o)
    assert s.max() <= 1.0, f"{what}: {s.max():.3f} BF16 steps at {np.unravel_index(s.argmax(), s.shape)}"
    cap = max(2, int(1e-3 * s.size))
    assert (s > 0.5).sum() <= cap, f"{what}: {(s > 0.5).sum()} elements beyond half a step"


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


@pytest.mark.parametrize("waves", [None, "1", "4", "k"])
@pytest.mark.parametrize("dims,B", [([64, 48, 40, 5], 37), ([512, 512, 512, 512, 5], 1024),
                                    ([100, 70, 3], 130), ([16, 16], 1)])
def test_forward_and_gradients(ctx, monkeypatch, dims, B, waves):
    """Forward output, loss and every gradient against the FP64 oracle at
    the same BF16 rounding points, with the matrix products' workgroups
    chosen by size or forced to one wavefront, to 2 x 2 wavefronts, or to
    four wavefronts splitting K (also where K has fewer than four steps)."""
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
    _assert_bf16_close(out.cpu().numpy(), oo, "output")
    assert abs(loss.item() - lo) <= 1e-3 * lo
    for l, (gW, gb) in enumerate(go):
        _assert_bf16_close(dW[l].cpu().numpy(), gW, f"dW[{l}]")
        _assert_bf16_close(db[l].cpu().numpy(), gb, f"db[{l}]")


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


def test_adam_kernel_elementwise(ctx):
    """The Adam kernel alone, element by element: three steps driven by the
    GPU's own gradients, against the oracle's FP64 Adam fed the same
    gradients.  Each parameter moves by about lr per step; the two sides
    differ only by FP32 rounding of the moments and of the parameter."""
    dims, B = [48, 40, 6], 96
    net, params, x, y, xb = _net(ctx, dims, B, 13)
    yt = torch.from_numpy(y).cuda()
    W0, b0 = net.get_params()
    p64 = [(Wq.cpu().numpy().astype(np.float64), bq.cpu().numpy().astype(np.float64))
           for Wq, bq in zip(W0, b0)]
    opt = omlp.Adam(p64)
    for step, lr in enumerate((1e-3, 2e-3, 5e-4)):
        net.backward(xb, yt)
        dW, db = net.get_grads()
        g64 = [(gW.cpu().numpy().astype(np.float64), gb.cpu().numpy().astype(np.float64))
               for gW, gb in zip(dW, db)]
        net.adam(lr)
        p64 = opt.step(p64, g64, lr)
        W, b = net.get_params()
        torch.cuda.synchronize()
        for l, (Wo, bo) in enumerate(p64):
            for got, want, name in ((W[l], Wo, "W"), (b[l], bo, "b")):
                got = got.cpu().numpy().astype(np.float64)
                # FP32 rounding of the stored parameter plus 1e-4 of the
                # step's size for the FP32 moments
                tol = 2.0 * np.spacing(np.abs(want).astype(np.float32)) + 1e-4 * lr
                assert np.all(np.abs(got - want) <= tol), f"step {step} {name}[{l}]"
        # continue both sides from the GPU's FP32 parameters
        p64 = [(Wq.cpu().numpy().astype(np.float64), bq.cpu().numpy().astype(np.float64))
               for Wq, bq in zip(W, b)]


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


@pytest.mark.parametrize("dims,B,steps,N", [([40, 32, 4], 64, 5, 330),
                                             ([512, 512, 512, 5], 1024, 3, 3 * 1024)])
def test_train_steps_equals_step_loop(ctx, dims, B, steps, N):
    """fjofc_mlp_train_steps against the same steps called one by one
    (backward on consecutive batches, Adam with each step's rate): the
    parameters, the Adam state's effect on a further step, and the summed
    loss are bitwise equal; rows beyond steps x B are not read."""
    rng = np.random.default_rng(B + steps)
    x = torch.from_numpy(rng.standard_normal((N, dims[0])).astype(np.float32)).cuda()
    x = x.to(torch.bfloat16)
    y = torch.from_numpy(rng.standard_normal((N, dims[-1])).astype(np.float32)).cuda()
    lrs = [1e-3 * (1 + 0.5 * np.cos(q)) for q in range(steps)]
    a, _, _, _, _ = _net(ctx, dims, B, 21)
    b, _, _, _, _ = _net(ctx, dims, B, 21)
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    acc = torch.zeros(1, dtype=torch.float64, device="cuda")
    for q in range(steps):
        a.backward(x[q * B:(q + 1) * B], y[q * B:(q + 1) * B], loss)
        a.adam(lrs[q])
        acc += loss
    tot = torch.zeros(1, dtype=torch.float64, device="cuda")
    b.train_steps(x, y, B, lrs, tot)
    # one more step each, so that the first and second moments must agree too
    a.backward(x[:B], y[:B])
    a.adam(2e-3)
    b.train_steps(x[:B], y[:B], B, [2e-3])
    Wa, ba = a.get_params()
    Wb, bb = b.get_params()
    torch.cuda.synchronize()
    assert tot.item() == acc.item()
    for l in range(len(Wa)):
        assert torch.equal(Wa[l], Wb[l]), f"W[{l}]"
        assert torch.equal(ba[l], bb[l]), f"b[{l}]"


def test_train_steps_rejects_bad_arguments(ctx):
    dims, B = [16, 8, 2], 10
    net, _, _, _, _ = _net(ctx, dims, B, 2)
    x = torch.zeros((25, 16), dtype=torch.bfloat16, device="cuda")
    y = torch.zeros((25, 2), dtype=torch.float32, device="cuda")
    W0, _ = net.get_params()
    for lrs in ([1e-3] * 3, [1e-3, -1e-3], [float("nan")]):
        with pytest.raises(fjofc.FjofcError):
            net.train_steps(x, y, B, lrs)
    with pytest.raises(fjofc.FjofcError):
        net.train_steps(x, y, B, [1e-3], beta1=1.0)
    with pytest.raises(fjofc.FjofcError):
        net.train_steps(x, y, B + 1, [1e-3])
    net.train_steps(x, y, B, [])
    W1, _ = net.get_params()
    for a, b in zip(W0, W1):
        assert torch.equal(a, b)


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


@pytest.mark.parametrize("N,F", [(1, 5), (37, 3), (1000, 300), (5003, 512)])
def test_feature_stats(ctx, N, F):
    """fjofc_mlp_feature_stats against the oracle's mean and sample SD; one
    constant column takes min_sd."""
    rng = np.random.default_rng(N + F)
    raw = (rng.standard_normal((N, F)) * rng.uniform(0.1, 5, F) + rng.uniform(-3, 3, F))
    raw = raw.astype(np.float32)
    raw[:, F // 2] = 1.25
    mu = torch.empty(F, dtype=torch.float32, device="cuda")
    isd = torch.empty_like(mu)
    fjofc.fjofc_mlp_feature_stats(ctx, torch.from_numpy(raw).cuda(), mu, isd, min_sd=1e-3)
    mo, io = omlp.feature_stats(raw, 1e-3)
    np.testing.assert_allclose(mu.cpu().numpy(), mo, rtol=1e-6, atol=1e-7 * np.abs(mo).max())
    np.testing.assert_allclose(isd.cpu().numpy(), io, rtol=2e-6)
    assert isd[F // 2].item() == pytest.approx(1e3, rel=1e-6)


@pytest.mark.parametrize("k,m,d", [(1, 1, 1), (37, 2, 5), (4096, 3, 2)])
def test_consensus_points(ctx, k, m, d):
    rng = np.random.default_rng(k)
    Y = rng.standard_normal((k, m, d)).astype(np.float32)
    out = torch.empty((k, d), dtype=torch.float32, device="cuda")
    fjofc.fjofc_oos_consensus(ctx, torch.from_numpy(Y).cuda(), out)
    np.testing.assert_allclose(out.cpu().numpy(), omlp.consensus(Y), rtol=1e-6, atol=1e-7)


@pytest.mark.parametrize("dims,B", [([64, 48, 40, 5], 37), ([512, 512, 512, 512, 5], 1024)])
def test_loss_only(ctx, dims, B):
    """fjofc_mlp_loss: the oracle's MSE at the BF16 rounding points; the
    stored gradients are not touched."""
    net, params, x, y, xb = _net(ctx, dims, B, 31 + B)
    yt = torch.from_numpy(y).cuda()
    net.backward(xb, yt)
    dW0, _ = net.get_grads()
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    net.loss(xb, yt, loss)
    dW1, _ = net.get_grads()
    torch.cuda.synchronize()
    lo, _, _ = omlp.loss_and_grads([(W.astype(np.float64), b.astype(np.float64))
                                    for W, b in params], x, y, bf16=True)
    assert abs(loss.item() - lo) <= 1e-3 * lo
    for a, b in zip(dW0, dW1):
        assert torch.equal(a, b)

