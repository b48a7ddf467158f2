"""Pins of the oracle's SwitchNet (CPU only): the forward pass and the loss
gradient against the same network built from torch.nn.Linear and
torch.nn.MultiheadAttention (4 heads, one token per node) in FP64, with and
without dropout; the BF16-rounded network within the rounding error of the
unrounded one; zero gradients of the query and key projections; the dropout
masks' statistics."""
import math

import numpy as np
import pytest
import torch

IN, H1, H2 = 10, 128, 256


def swn_params(oracle_mod, seed):
    """He-normal weights (W[in][out]), small biases, in the oracle's layout."""
    rng = np.random.default_rng(seed)
    parts = []
    for ni, no in [(IN, H1), (H1, H2)] + [(H2, H2)] * 4:
        parts.append(rng.normal(0, math.sqrt(2 / ni), ni * no))
        parts.append(rng.normal(0, 0.05, no))
    parts.append(rng.normal(0, math.sqrt(1 / H2), H2))
    parts.append(rng.normal(0, 0.05, 1))
    p = np.concatenate(parts)
    assert p.size == oracle_mod.swn_nparam()
    return p


def _split(p):
    out, o = [], 0
    for ni, no in [(IN, H1), (H1, H2)] + [(H2, H2)] * 4:
        out.append((p[o:o + ni * no].reshape(ni, no), p[o + ni * no:o + ni * no + no]))
        o += ni * no + no
    out.append((p[o:o + H2], p[o + H2:o + H2 + 1]))
    return out


def _torch_net(p, rnd):
    """The network on torch FP64 tensors sliced from p: linear blocks and
    torch's multi-head attention forward (4 heads) over a length-1 sequence."""
    bf = (lambda t: t.to(torch.bfloat16).to(torch.float64)) if rnd else (lambda t: t)
    (W1, b1), (W2, b2), (Wq, bq), (Wk, bk), (Wv, bv), (Wo, bo), (wh, bh) = _split(p)

    def run(x, mask=None):
        x = bf(x)
        h1 = torch.relu(x @ bf(W1) + b1) + torch.nn.functional.pad(x, (0, H1 - IN))
        h2 = torch.relu(h1 @ bf(W2) + b2) + torch.nn.functional.pad(h1, (0, H2 - H1))
        if mask is not None:
            h2 = h2 * mask
        t = h2[:, None, :]
        a, _ = torch.nn.functional.multi_head_attention_forward(
            t.transpose(0, 1), t.transpose(0, 1), t.transpose(0, 1), H2, 4,
            torch.cat([bf(Wq).T, bf(Wk).T, bf(Wv).T]), torch.cat([bq, bk, bv]), None, None, False, 0.0,
            bf(Wo).T, bo, training=False, need_weights=False)
        a = a.transpose(0, 1)[:, 0, :]
        return a @ bf(wh) + bh[0]
    return run


def _mask(oracle_mod, n, step):
    return np.stack([oracle_mod.swn_mask(77, v, step, 0) for v in range(n)])


@pytest.fixture
def no_rounding(oracle_mod):
    oracle_mod.cnn_set_rounding(False)
    yield
    oracle_mod.cnn_set_rounding(True)


@pytest.mark.parametrize("dropout", [False, True])
def test_forward_matches_torch_attention(oracle_mod, no_rounding, dropout):
    p = swn_params(oracle_mod, 1)
    x = np.random.default_rng(2).normal(0, 1, (37, IN))
    mask = _mask(oracle_mod, 37, 4) if dropout else None
    got = oracle_mod.swn_forward(p, x, mask=mask)
    ref = _torch_net(torch.tensor(p), False)(torch.tensor(x), None if mask is None else torch.tensor(mask))
    np.testing.assert_allclose(got, ref.detach().numpy(), rtol=1e-10, atol=1e-10)


def test_rounded_forward_within_bf16_error(oracle_mod):
    """Rounding the stored activations (h1, h2, v, a) on top of BF16 weights
    moves each logit by a few BF16 steps of the values summed into it."""
    p = swn_params(oracle_mod, 3)
    x = np.random.default_rng(4).normal(0, 1, (200, IN))
    got = oracle_mod.swn_forward(p, x)
    ref = _torch_net(torch.tensor(p), True)(torch.tensor(x)).detach().numpy()
    rms = np.sqrt((ref ** 2).mean())
    err = np.abs(got - ref) / rms
    assert np.median(err) < 2 ** -8 and err.max() < 2 ** -5
    assert not np.array_equal(got, ref)


@pytest.mark.parametrize("dropout", [False, True])
def test_loss_and_gradient_match_autograd(oracle_mod, no_rounding, dropout):
    p = swn_params(oracle_mod, 5)
    rng = np.random.default_rng(6)
    n = 29
    x = rng.normal(0, 1, (n, IN))
    y = (rng.uniform(0, 1, n) > 0.5).astype(np.float64)
    e = rng.uniform(0, 1, n)
    mask = _mask(oracle_mod, n, 9) if dropout else None
    loss, g = oracle_mod.swn_loss_grad(p, x, y, e, lam=0.1, mask=mask)
    pt = torch.tensor(p, requires_grad=True)
    lg = _torch_net(pt, False)(torch.tensor(x), None if mask is None else torch.tensor(mask))
    pr = torch.sigmoid(lg)
    lt = (torch.nn.functional.binary_cross_entropy_with_logits(lg, torch.tensor(y), reduction="none") +
          0.1 * (1 - pr) * torch.tensor(e)).mean()
    lt.backward()
    assert loss == pytest.approx(lt.item(), rel=1e-11)
    gt = pt.grad.numpy()
    np.testing.assert_allclose(g, gt, rtol=1e-8, atol=1e-12 * np.abs(gt).max())
    # query and key projections: exactly no gradient (softmax over one key)
    o = IN * H1 + H1 + H1 * H2 + H2
    qk = slice(o, o + 2 * (H2 * H2 + H2))
    assert np.all(g[qk] == 0.0) and np.abs(gt[qk]).max() < 1e-14


def test_dropout_masks(oracle_mod):
    m = np.stack([oracle_mod.swn_mask(5, v, 3, 2) for v in range(2000)])
    assert set(np.unique(m)) <= {0.0, 256 / 205}
    rate = (m == 0).mean()
    sigma = math.sqrt(51 / 256 * (1 - 51 / 256) / m.size)
    assert abs(rate - 51 / 256) < 4 * sigma
    assert (oracle_mod.swn_mask(5, 17, 3, 2) == m[17]).all()
    assert not (oracle_mod.swn_mask(5, 17, 3, 1) == m[17]).all()
    assert not (oracle_mod.swn_mask(5, 17, 4, 2) == m[17]).all()
