"""Pins of the oracle's next-state surrogate (CPU only): the forward pass
against the same network written with torch's conv3d in FP64, the loss
(Huber and energy term) and its gradient against torch autograd, with and
without dropout, and the dropout masks' statistics."""
import math

import numpy as np
import pytest
import torch

CIN = (10, 13, 32, 64, 128, 32)
COUT = (13, 32, 64, 128, 32, 10)
RES = (1, 1, 1, 0, 0, 0)
RELU = (1, 1, 1, 1, 1, 0)


def sp_params(oracle_mod, seed, scale=1.0):
    """He-normal weights, small biases, in the oracle's parameter layout."""
    rng = np.random.default_rng(seed)
    p = np.zeros(oracle_mod.sp_nparam())
    o = 0
    for ci, co in zip(CIN, COUT):
        n = 27 * ci * co
        p[o:o + n] = rng.normal(0, scale * math.sqrt(2 / (27 * ci)), n)
        p[o + n:o + n + co] = rng.normal(0, 0.05, co)
        o += n + co
    assert o == p.size
    return p


def _torch_forward(p, x, rnd, mask=None):
    """The network with torch (FP64): conv3d with padding 1 on channels-first
    tensors, weights rearranged to [co, ci, kz, ky, kx]; the residual copies
    the block input into the first output channels."""
    bf = (lambda t: t.to(torch.bfloat16).to(torch.float64)) if rnd else (lambda t: t)
    a = bf(x.permute(0, 4, 1, 2, 3))
    o = 0
    for l, (ci, co) in enumerate(zip(CIN, COUT)):
        n = 27 * ci * co
        W = p[o:o + n].reshape(3, 3, 3, ci, co).permute(4, 3, 0, 1, 2)
        b = p[o + n:o + n + co]
        o += n + co
        z = torch.nn.functional.conv3d(a, bf(W), b, padding=1)
        h = torch.relu(z) if RELU[l] else z
        if RES[l]:
            h = h + torch.nn.functional.pad(a, (0, 0, 0, 0, 0, 0, 0, co - ci))
        if l == len(CIN) - 1:
            a = h
            break
        if l == 1 and mask is not None:
            h = h * mask.permute(0, 4, 1, 2, 3)
        a = bf(h)
    return a.permute(0, 2, 3, 4, 1)


def _torch_loss(pred, y, mean, std, delta, lam):
    hub = torch.nn.functional.huber_loss(pred, y, delta=delta)
    e_p = ((pred[..., :6] * std[:6] + mean[:6]) ** 2).sum(dim=(1, 2, 3, 4))
    e_t = ((y[..., :6] * std[:6] + mean[:6]) ** 2).sum(dim=(1, 2, 3, 4))
    return hub + lam * (((e_p - e_t) / e_t) ** 2).mean()


def test_forward_matches_torch(oracle_mod):
    p = sp_params(oracle_mod, 1)
    x = np.random.default_rng(2).normal(0, 1, (2, 5, 4, 6, 10))
    got = oracle_mod.sp_forward(p, x)
    ref = _torch_forward(torch.tensor(p), torch.tensor(x), True).numpy()
    assert got.shape == x.shape
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)


def test_forward_with_dropout_rounds_once(oracle_mod):
    """BF16 rounding with dropout: block 2's output is scaled, then rounded."""
    p = sp_params(oracle_mod, 3)
    shape = (1, 4, 5, 3)
    x = np.random.default_rng(4).normal(0, 1, shape + (10,))
    mask = np.stack([oracle_mod.sp_mask(11, v, 2, 0) for v in range(int(np.prod(shape)))]).reshape(shape + (32,))
    got = oracle_mod.sp_forward(p, x, mask=mask)
    ref = _torch_forward(torch.tensor(p), torch.tensor(x), True, torch.tensor(mask)).numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-10, atol=1e-10)
    assert not np.allclose(got, oracle_mod.sp_forward(p, x), atol=1e-6)


@pytest.fixture
def no_rounding(oracle_mod):
    oracle_mod.cnn_set_rounding(False)
    yield
    oracle_mod.cnn_set_rounding(True)


@pytest.mark.parametrize("dropout", [False, True])
def test_loss_and_gradient_match_autograd(oracle_mod, no_rounding, dropout):
    rng = np.random.default_rng(3)
    p = sp_params(oracle_mod, 4)
    shape = (2, 4, 3, 5)
    x = rng.normal(0, 1, shape + (10,))
    y = rng.normal(0, 0.02, shape + (10,)) + 0.5 * x       # a target near the input
    mean = rng.normal(0, 0.1, 10); std = rng.uniform(0.5, 2.0, 10)
    mask = None
    if dropout:
        mask = np.stack([oracle_mod.sp_mask(99, v, 7, 0) for v in range(int(np.prod(shape)))]).reshape(shape + (32,))
    loss, g = oracle_mod.sp_loss_grad(p, x, y, mean, std, delta=0.01, lam=0.1, mask=mask)
    pt = torch.tensor(p, requires_grad=True)
    pred = _torch_forward(pt, torch.tensor(x), False, None if mask is None else torch.tensor(mask))
    lt = _torch_loss(pred, torch.tensor(y), torch.tensor(mean), torch.tensor(std), 0.01, 0.1)
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-12)
    np.testing.assert_allclose(g, pt.grad.numpy(), rtol=1e-8, atol=1e-12 * np.abs(g).max())


def test_huber_branches(oracle_mod, no_rounding):
    # every residual beyond delta: the loss is linear in the error and the
    # gradient of the output is +-delta / count (read through the last bias)
    p = sp_params(oracle_mod, 5)
    x = np.zeros((1, 2, 2, 2, 10))
    pred = oracle_mod.sp_forward(p, x)
    y = pred - 0.5
    loss, g = oracle_mod.sp_loss_grad(p, x, y, np.zeros(10), np.ones(10), delta=0.01, lam=0.0)
    assert loss == pytest.approx(0.01 * (0.5 - 0.005), rel=1e-12)
    gb = g[-10:]      # bias of the output layer: mean of dL/dpred over voxels
    np.testing.assert_allclose(gb, 0.01 / 10, rtol=1e-12)


def test_dropout_masks(oracle_mod):
    m = np.stack([oracle_mod.sp_mask(5, v, 3, 1) for v in range(4000)])
    kept = (m > 0).mean()
    # drop probability 26/256, binomial over 128000 channel draws
    assert abs((1 - kept) - 26 / 256) < 5 * math.sqrt(26 / 256 * 230 / 256 / m.size)
    assert set(np.unique(m)) == {0.0, 256 / 230}
    assert (oracle_mod.sp_mask(5, 17, 3, 1) == m[17]).all()
    assert not (oracle_mod.sp_mask(5, 17, 4, 1) == m[17]).all()
