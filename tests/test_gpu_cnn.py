"""GPU parity of the switch network (BF16 matrix-core forward, backward and
AdamW) and of the learned switch mode, against the FP64 oracle."""
import math

import numpy as np
import pytest

from paper_2510_11174_amd import configs
from tests.test_oracle_cnn import _params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _crops(seed, B=2, D=24, H=24, W=24):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (B, D, H, W, 8)).astype(np.float32)
    n = (B, D - 8, H - 8, W - 8)
    y = (rng.uniform(0, 1, n) > 0.7).astype(np.float32)
    e = rng.uniform(0, 1, n).astype(np.float32)
    return x, y, e


def _dev(*arrs):
    import torch
    return [torch.tensor(a, device="cuda") for a in arrs]


def _net(hk, oracle_mod, seed):
    # parameters exactly representable in FP32: both sides start from the same values
    p = _params(oracle_mod, seed).astype(np.float32).astype(np.float64)
    c = hk.CNN(seed=77)
    c.set_params(p)
    return c, p


def test_forward(hk, oracle_mod):
    # ragged sizes: 24^3 crops (16^3 outputs) and a 13 x 20 x 29 box
    for shape in [(2, 24, 24, 24), (1, 13, 20, 29)]:
        print("case: cnn forward", shape, flush=True)
        c, p = _net(hk, oracle_mod, 11)
        x, _, _ = _crops(3, *shape)
        (xd,) = _dev(x)
        got = c.forward(xd).cpu().numpy()
        ref = oracle_mod.cnn_forward(p, x.astype(np.float64))
        rms = np.sqrt((ref ** 2).mean())
        ae = np.abs(got - ref) / rms
        rl2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
        dec = ((got > 0) != (ref > 0)).mean()
        print("logits: rel L2 %.2e; |err|/rms median %.2e 99th %.2e max %.2e; sign flips %.2e" % (
            rl2, np.median(ae), np.percentile(ae, 99), ae.max(), dec))
        assert np.median(ae) < 1e-5 and rl2 < 1e-2 and np.percentile(ae, 99) < 3e-2


@pytest.mark.parametrize("dropout", [False, True])
def test_loss_and_gradient(hk, oracle_mod, dropout):
    print("case: cnn gradient dropout=%s" % dropout, flush=True)
    c, p = _net(hk, oracle_mod, 12)
    x, y, e = _crops(4, B=2, D=20, H=18, W=22)
    xd, yd, ed = _dev(x, y, e)
    step = 5 if dropout else -1
    loss, g = c.loss_grad(xd, yd, ed, lam=0.1, mask_step=step)
    mask = None
    if dropout:
        n = y.size
        mask = np.stack([oracle_mod.cnn_mask(77, v, step, 0) for v in range(n)]).reshape(y.shape + (32,))
    lo, go = oracle_mod.cnn_loss_grad(p, x.astype(np.float64), y.astype(np.float64), e.astype(np.float64),
                                      lam=0.1, mask=mask)
    print("loss %.8f / %.8f" % (loss, lo))
    assert loss == pytest.approx(lo, rel=1e-4)
    # per layer relative L2 of the gradient (BF16 pre-activation gradients on the GPU)
    offs = np.cumsum([0, 27 * 8 * 32 + 32] + [27 * 32 * 32 + 32] * 3 + [33])
    for l in range(5):
        a, b = g[offs[l]:offs[l + 1]], go[offs[l]:offs[l + 1]]
        rl = np.linalg.norm(a - b) / np.linalg.norm(b)
        print("layer %d gradient rel L2 %.2e" % (l, rl))
        assert rl <= 1e-2


def test_adamw_steps(hk, oracle_mod):
    print("case: cnn AdamW steps", flush=True)
    c, p = _net(hk, oracle_mod, 13)
    x, y, e = _crops(5, B=2, D=18, H=18, W=18)
    xd, yd, ed = _dev(x, y, e)
    m = np.zeros_like(p); v = np.zeros_like(p); po = p.copy()
    for t in range(1, 4):
        c.train_step(xd, yd, ed, lr=1e-3, lam=0.1, dropout=False)
        _, go = oracle_mod.cnn_loss_grad(po, x.astype(np.float64), y.astype(np.float64),
                                         e.astype(np.float64), lam=0.1)
        oracle_mod.cnn_adamw(po, go, m, v, t)
    pg = c.get_params().astype(np.float64)
    # AdamW moves each parameter by about lr per step; compare the moves
    dg, do = pg - p, po - p
    rl = np.linalg.norm(dg - do) / np.linalg.norm(do)
    print("parameter update rel L2 %.2e" % rl)
    assert rl <= 2e-2


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_cnn_switch_mode(hk, oracle_mod, prec):
    # the learned switch inside the step: same network and statistics on both
    # sides; maps compared node by node after a few evaluations.  The network
    # runs in BF16 in both builds; the build sets the precision of the fields
    # and moments it reads (a node whose mean p or spread sits at a decision
    # threshold may go either way: at most 2e-3 of the nodes)
    cfg = configs.plain_hybrid(24, 12, 12, mode="cnn")
    cfg["run"]["switch_every"] = 10
    print("case: cnn switch", cfg["name"], prec, flush=True)
    # statistics and head bias chosen so that the map is mixed (about 80% kinetic)
    p = _params(oracle_mod, 14, scale=0.5)
    p[-1] = -0.8
    p = p.astype(np.float32).astype(np.float64)
    mean = np.array([0, 0, 0, 0, 0, 0, 0.01, 0], np.float32)
    std = np.array([0.01, 0.01, 0.01, 0.01, 0.01, 0.01, 1e-4, 1e-3], np.float32)
    g = hk.Sim(cfg, precision=prec); o = oracle_mod.Oracle(cfg)
    c = hk.CNN(seed=cfg["run"]["seed"], precision=prec)
    c.set_params(p); c.set_norm(mean, std)
    g.set_cnn(c)
    o.set_cnn(p, mean.astype(np.float64), std.astype(np.float64))
    for n in range(4):
        g.step(10); o.step(10)
        mg, mo = g.get_switch(), o.get_switch()
        dg, do = g.diagnostics(), o.diagnostics()
        mis = (mg != mo).mean()
        print("step %d kinetic %.3f / %.3f mismatch %.2e fallback %.3f / %.3f" % (
            10 * (n + 1), mg.mean(), mo.mean(), mis, dg["fallback_fraction"], do["fallback_fraction"]))
        assert mis <= 2e-3
        assert abs(dg["fallback_fraction"] - do["fallback_fraction"]) <= 2e-3
        if n >= 1:
            assert 0.05 < mo.mean() < 0.95
