"""Pins of the FP64 MLP oracle: bfloat16 rounding against torch's
conversion, GELU against torch's exact GELU, gradients against central
finite differences, Adam against torch.optim.Adam."""
import numpy as np
import pytest
import torch

from oracle import mlp


def test_bf16_round_matches_torch():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(10000) * 10.0 ** rng.integers(-6, 6, 10000),
                        [0.0, -0.0, 1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -9, -1.5 - 2 ** -8]])
    ref = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(mlp.bf16_round(x), ref)
    # ties to even: 1 + 2^-8 lies halfway between 1 and 1 + 2^-7
    assert mlp.bf16_round(1.0 + 2 ** -8) == 1.0


def test_gelu_matches_torch_exact_gelu():
    z = np.linspace(-8, 8, 1001)
    ref = torch.nn.functional.gelu(torch.from_numpy(z), approximate="none").numpy()
    np.testing.assert_allclose(mlp.gelu(z), ref, rtol=1e-14, atol=1e-15)
    zt = torch.from_numpy(z).requires_grad_(True)
    torch.nn.functional.gelu(zt, approximate="none").sum().backward()
    np.testing.assert_allclose(mlp.gelu_grad(z), zt.grad.numpy(), rtol=1e-12, atol=1e-14)


def test_gradients_match_finite_differences():
    dims = [7, 6, 5, 3]
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.1)
              for W, b in mlp.init_params(dims, 1)]
    rng = np.random.default_rng(2)
    x = rng.standard_normal((9, dims[0]))
    y = rng.standard_normal((9, dims[-1]))
    _, grads, _ = mlp.loss_and_grads(params, x, y, bf16=False)
    h = 1e-6
    for l in range(len(params)):
        for j in range(2):
            p = params[l][j]
            num = np.zeros_like(p)
            for idx in np.ndindex(p.shape):
                saved = p[idx]
                p[idx] = saved + h
                lp, _, _ = mlp.loss_and_grads(params, x, y, bf16=False)
                p[idx] = saved - h
                lm, _, _ = mlp.loss_and_grads(params, x, y, bf16=False)
                p[idx] = saved
                num[idx] = (lp - lm) / (2 * h)
            np.testing.assert_allclose(grads[l][j], num, rtol=1e-6, atol=1e-9)


def test_gradients_match_torch_autograd():
    dims = [16, 12, 12, 4]
    params = [(W.astype(np.float64), b.astype(np.float64))
              for W, b in mlp.init_params(dims, 3)]
    rng = np.random.default_rng(4)
    x = rng.standard_normal((10, dims[0]))
    y = rng.standard_normal((10, dims[-1]))
    loss, grads, _ = mlp.loss_and_grads(params, x, y, bf16=False)
    tp = [(torch.tensor(W, requires_grad=True), torch.tensor(b, requires_grad=True)) for W, b in params]
    h = torch.tensor(x)
    for l, (W, b) in enumerate(tp):
        h = h @ W + b
        if l < len(tp) - 1:
            h = torch.nn.functional.gelu(h)
    tl = ((h - torch.tensor(y)) ** 2).mean()
    tl.backward()
    assert loss == pytest.approx(tl.item(), rel=1e-13)
    for (gW, gb), (W, b) in zip(grads, tp):
        np.testing.assert_allclose(gW, W.grad.numpy(), rtol=1e-11, atol=1e-14)
        np.testing.assert_allclose(gb, b.grad.numpy(), rtol=1e-11, atol=1e-14)


def test_adam_matches_torch():
    dims = [5, 4, 2]
    params = [(W.astype(np.float64), b.astype(np.float64) + 0.3) for W, b in mlp.init_params(dims, 5)]
    rng = np.random.default_rng(6)
    opt = mlp.Adam(params)
    tp = [torch.tensor(a) for W, b in params for a in (W, b)]
    for t in tp:
        t.requires_grad_(True)
    topt = torch.optim.Adam(tp, lr=1e-2, betas=(0.9, 0.999), eps=1e-8)
    cur = params
    for _ in range(5):
        grads = [(rng.standard_normal(W.shape), rng.standard_normal(b.shape)) for W, b in cur]
        cur = opt.step(cur, grads, 1e-2)
        for t, g in zip(tp, [a for gw in grads for a in gw]):
            t.grad = torch.tensor(g)
        topt.step()
    for (W, b), tW, tb in zip(cur, tp[0::2], tp[1::2]):
        np.testing.assert_allclose(W, tW.detach().numpy(), rtol=1e-12, atol=1e-14)
        np.testing.assert_allclose(b, tb.detach().numpy(), rtol=1e-12, atol=1e-14)
