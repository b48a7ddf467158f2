"""Pins of the oracle's switch network (CPU only): the forward pass against
torch's conv3d in FP64, gradients against finite differences and against
torch autograd, AdamW against torch.optim.AdamW, and the dropout masks'
statistics."""
import math

import numpy as np
import pytest
import torch

NC = 32


def _layers(params):
    """Split the parameter vector into (W[27, cin, 32], b[32]) per layer and the head."""
    out, o = [], 0
    for cin in (8, 32, 32, 32):
        n = 27 * cin * NC
        out.append((params[o:o + n].reshape(27, cin, NC), params[o + n:o + n + NC]))
        o += n + NC
    return out, params[o:o + NC], params[o + NC]


def _torch_forward(params, x, rnd):
    """The same network written with torch (FP64): conv3d on channels-first
    tensors, weights rearranged to [co, ci, kz, ky, kx]."""
    bf = (lambda t: t.to(torch.bfloat16).to(torch.float64)) if rnd else (lambda t: t)
    layers, wh, bh = _layers(params)
    a = bf(x.permute(0, 4, 1, 2, 3))
    for W, b in layers:
        w = bf(W.reshape(3, 3, 3, W.shape[1], NC).permute(4, 3, 0, 1, 2))   # [t=kz,ky,kx]
        z = torch.nn.functional.conv3d(a, w, b)
        a = bf(0.5 * z * (1 + torch.erf(z / math.sqrt(2))))
    return torch.einsum("bcdhw,c->bdhw", a, bf(wh)) + bh


def _params(oracle_mod, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle_mod.cnn_nparam())
    o = 0
    for cin in (8, 32, 32, 32):
        n = 27 * cin * NC
        p[o:o + n] = rng.normal(0, scale * math.sqrt(2 / (27 * cin)), n)
        p[o + n:o + n + NC] = rng.normal(0, 0.1, NC)
        o += n + NC
    p[o:o + NC] = rng.normal(0, 0.3, NC)
    p[o + NC] = 0.05
    return p


def test_forward_matches_torch_conv3d(oracle_mod):
    p = _params(oracle_mod, 1)
    x = np.random.default_rng(2).normal(0, 1, (2, 11, 10, 12, 8))
    got = oracle_mod.cnn_forward(p, x)
    ref = _torch_forward(torch.tensor(p), torch.tensor(x), True).numpy()
    assert got.shape == (2, 3, 2, 4)
    np.testing.assert_allclose(got, ref, rtol=1e-12, atol=1e-12)


def test_forward_bf16_rounding_is_round_to_nearest_even(oracle_mod):
    for v in [1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, -(1.0 + 2 ** -8), 3.14159, 1e-20, 65504.3]:
        ref = float(torch.tensor(v, dtype=torch.float64).to(torch.bfloat16).to(torch.float64))
        assert oracle_mod.bf16(v) == ref


@pytest.fixture
def no_rounding(oracle_mod):
    oracle_mod.cnn_set_rounding(False)
    yield
    oracle_mod.cnn_set_rounding(True)


def _batch(seed, B=2, D=10):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (B, D, D, D, 8))
    n = D - 8
    y = (rng.uniform(0, 1, (B, n, n, n)) > 0.6).astype(float)
    e = rng.uniform(0, 1, (B, n, n, n))
    return x, y, e


def test_gradient_finite_differences(oracle_mod, no_rounding):
    p = _params(oracle_mod, 3)
    x, y, e = _batch(4)
    loss, g = oracle_mod.cnn_loss_grad(p, x, y, e, lam=0.1)
    rng = np.random.default_rng(5)
    layers_end = np.cumsum([27 * 8 * NC + NC] + [27 * 32 * NC + NC] * 3 + [NC + 1])
    idx = list(rng.integers(0, p.size, 12)) + [int(v) - 1 for v in layers_end]   # biases too
    for i in idx:
        h = 1e-5 * max(1.0, abs(p[i]))
        pp = p.copy(); pp[i] += h
        pm = p.copy(); pm[i] -= h
        lp, _ = oracle_mod.cnn_loss_grad(pp, x, y, e, lam=0.1)
        lm, _ = oracle_mod.cnn_loss_grad(pm, x, y, e, lam=0.1)
        fd = (lp - lm) / (2 * h)
        assert g[i] == pytest.approx(fd, rel=1e-6, abs=1e-11), i


def test_gradient_matches_torch_autograd(oracle_mod, no_rounding):
    p = _params(oracle_mod, 6)
    x, y, e = _batch(7, B=1, D=11)
    mask = np.stack([oracle_mod.cnn_mask(99, v, 3, 0) for v in range(27)]).reshape(1, 3, 3, 3, NC)
    loss, g = oracle_mod.cnn_loss_grad(p, x, y, e, lam=0.1, mask=mask)
    pt = torch.tensor(p, requires_grad=True)
    layers, wh, bh = _layers(pt)
    a = torch.tensor(x).permute(0, 4, 1, 2, 3)
    for W, b in layers:
        w = W.reshape(3, 3, 3, W.shape[1], NC).permute(4, 3, 0, 1, 2)
        z = torch.nn.functional.conv3d(a, w, b)
        a = 0.5 * z * (1 + torch.erf(z / math.sqrt(2)))
    a = a * torch.tensor(mask).permute(0, 4, 1, 2, 3)
    lg = torch.einsum("bcdhw,c->bdhw", a, wh) + bh
    pr = torch.sigmoid(lg)
    yt, et = torch.tensor(y), torch.tensor(e)
    lt = (torch.nn.functional.binary_cross_entropy_with_logits(lg, yt, reduction="none")
          + 0.1 * (1 - pr) * et).mean()
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-9, atol=1e-14)


def test_adamw_matches_torch(oracle_mod):
    rng = np.random.default_rng(8)
    p = rng.normal(0, 1, 50); m = np.zeros(50); v = np.zeros(50)
    pt = torch.tensor(p.copy(), requires_grad=True)
    opt = torch.optim.AdamW([pt], lr=1e-3, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    for t in range(1, 4):
        g = rng.normal(0, 1, 50)
        oracle_mod.cnn_adamw(p, g, m, v, t)
        opt.zero_grad(); pt.grad = torch.tensor(g); opt.step()
        np.testing.assert_allclose(p, pt.detach().numpy(), rtol=1e-13, atol=1e-15)


def test_dropout_masks(oracle_mod):
    m = np.stack([oracle_mod.cnn_mask(2025, node, 0, s) for node in range(200) for s in range(16)])
    kept = m > 0
    n = kept.size
    p_drop = 26 / 256
    assert abs((~kept).mean() - p_drop) < 4 * math.sqrt(p_drop * (1 - p_drop) / n)
    assert np.allclose(m[kept], 256 / 230)
    assert abs(m.mean() - 1.0) < 0.01
    # masks depend on the node, the evaluation and the sample
    assert not np.array_equal(oracle_mod.cnn_mask(2025, 1, 0, 0), oracle_mod.cnn_mask(2025, 1, 1, 0))
    assert not np.array_equal(oracle_mod.cnn_mask(2025, 1, 0, 0), oracle_mod.cnn_mask(2025, 1, 0, 1))
