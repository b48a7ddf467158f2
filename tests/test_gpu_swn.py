"""GPU parity of the paper's SwitchNet (BF16 matrix-core linear layers, the
single-token attention, loss, backward and AdamW) against the FP64 oracle.

Same bar as the other networks: both sides use the same BF16 inputs and
weights, the GPU sums in FP32 and rounds stored activations to BF16, so a
sum that lands on the other side of a rounding boundary moves by one BF16
step.  Logits: median error at FP32 level, relative L2 below 1e-2; gradients:
per-layer relative L2 below 1e-2 (the GPU also rounds the backward signals to
BF16).
"""
import numpy as np
import pytest

from tests.test_oracle_swn import H1, H2, IN, swn_params

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _net(hk, oracle_mod, seed):
    p = swn_params(oracle_mod, seed).astype(np.float32).astype(np.float64)
    c = hk.SwitchNet(seed=77)
    c.set_params(p)
    return c, p


def _data(seed, n):
    rng = np.random.default_rng(seed)
    x = rng.normal(0, 1, (n, IN)).astype(np.float32)
    y = (rng.uniform(0, 1, n) > 0.6).astype(np.float32)
    e = rng.uniform(0, 1, n).astype(np.float32)
    return x, y, e


def _dev(*arrs):
    import torch
    return [torch.tensor(a, device="cuda") for a in arrs]


def _mask(oracle_mod, n, step, sample):
    return np.stack([oracle_mod.swn_mask(77, v, step, sample) for v in range(n)])


def _compare(got, ref, what):
    rms = np.sqrt((ref ** 2).mean())
    ae = np.abs(got - ref) / rms
    rl2 = np.linalg.norm(got - ref) / np.linalg.norm(ref)
    print("%s: rel L2 %.2e; |err|/rms median %.2e 99th %.2e max %.2e" % (
        what, rl2, np.median(ae), np.percentile(ae, 99), ae.max()))
    assert np.median(ae) < 1e-3 and rl2 < 1e-2 and np.percentile(ae, 99) < 3e-2


# n = 1000 ends in a partial 16-node row tile, n = 37 in one of 5 nodes
@pytest.mark.parametrize("n,step,sample", [(1000, -1, 0), (37, -1, 0), (1000, 3, 0), (333, 3, 5)])
def test_forward(hk, oracle_mod, n, step, sample):
    print("case: swn forward n=%d step=%d sample=%d" % (n, step, sample), flush=True)
    c, p = _net(hk, oracle_mod, 31)
    x, _, _ = _data(1, n)
    (xd,) = _dev(x)
    got = c.forward(xd, mask_step=step, sample=sample).cpu().numpy()
    mask = _mask(oracle_mod, n, step, sample) if step >= 0 else None
    ref = oracle_mod.swn_forward(p, x.astype(np.float64), mask=mask)
    _compare(got, ref, "logits")


def _slices():
    o, out = 0, []
    names = ["W1", "b1", "W2", "b2", "Wq", "bq", "Wk", "bk", "Wv", "bv", "Wo", "bo"]
    sizes = [IN * H1, H1, H1 * H2, H2] + [H2 * H2, H2] * 4
    for nm, sz in zip(names, sizes):
        out.append((nm, slice(o, o + sz)))
        o += sz
    out.append(("wh", slice(o, o + H2)))
    out.append(("bh", slice(o + H2, o + H2 + 1)))
    return out


@pytest.mark.parametrize("dropout", [False, True])
def test_loss_and_gradient(hk, oracle_mod, dropout):
    n = 512
    print("case: swn gradient dropout=%s n=%d" % (dropout, n), flush=True)
    c, p = _net(hk, oracle_mod, 32)
    x, y, e = _data(2, n)
    xd, yd, ed = _dev(x, y, e)
    step = 6 if dropout else -1
    loss, g = c.loss_grad(xd, yd, ed, lam=0.1, mask_step=step)
    mask = _mask(oracle_mod, n, step, 0) if dropout else None
    lo, go = oracle_mod.swn_loss_grad(p, x.astype(np.float64), y.astype(np.float64), e.astype(np.float64),
                                      lam=0.1, mask=mask)
    print("loss %.8f / %.8f" % (loss, lo))
    assert loss == pytest.approx(lo, rel=1e-4)
    for nm, s in _slices():
        if nm in ("Wq", "bq", "Wk", "bk"):
            assert np.all(g[s] == 0.0) and np.all(go[s] == 0.0)
            continue
        rl = np.linalg.norm(g[s] - go[s]) / np.linalg.norm(go[s])
        print("%s gradient rel L2 %.2e" % (nm, rl))
        assert rl <= 1e-2


def test_adamw_steps(hk, oracle_mod):
    n = 256
    print("case: swn AdamW steps n=%d" % n, flush=True)
    c, p = _net(hk, oracle_mod, 33)
    x, y, e = _data(3, n)
    xd, yd, ed = _dev(x, y, e)
    m = np.zeros_like(p); v = np.zeros_like(p); po = p.copy()
    losses, g1 = [], None
    for t in range(1, 4):
        losses.append(c.train_step(xd, yd, ed, lr=1e-4, lam=0.1, dropout=False))
        _, go = oracle_mod.swn_loss_grad(po, x.astype(np.float64), y.astype(np.float64), e.astype(np.float64),
                                         lam=0.1)
        g1 = go if g1 is None else g1
        oracle_mod.cnn_adamw(po, go, m, v, t, lr=1e-4)
    pg = c.get_params().astype(np.float64)
    dg, do = pg - p, po - p
    # AdamW's first moves are about lr times the gradient's sign: compare
    # where the oracle's gradient is clearly nonzero (query and key
    # projections have none and move by weight decay only)
    sure = np.abs(g1) > 0.05 * np.sqrt((g1 ** 2).mean())
    rl = np.linalg.norm((dg - do)[sure]) / np.linalg.norm(do[sure])
    print("losses %s; clear gradients %.3f; update rel L2 %.2e" % (losses, sure.mean(), rl))
    assert rl <= 2e-2
    assert losses[-1] < losses[0]


def test_rejects_bad_sizes(hk, oracle_mod):
    import torch
    c, _ = _net(hk, oracle_mod, 34)
    x = torch.zeros((12, IN), device="cuda")
    y = torch.zeros(12, device="cuda")
    with pytest.raises(hk.HKError):
        c.loss_grad(x, y, y)            # training needs n % 8 == 0
    with pytest.raises(hk.HKError):
        c.forward(x, mask_step=0, sample=16)


def test_switchnet_against_cnn_on_simulation_labels(hk):
    """The A/B of the two learned switches on the same all-PIC runs: the
    paper's per-node SwitchNet (node state only) and the 3D CNN (a 9^3
    neighbourhood), both trained by the library, scored by the AUC of the
    future-kinetic label on a held-out run."""
    from paper_2510_11174_amd import configs
    from paper_2510_11174_amd import train as T
    from tests import switch_data as SD

    def cfg(seed, a0):
        c = configs.plain_hybrid(32, 16, 16, mode="all_pic", seed=seed)
        c["laser"]["a0"] = a0
        return c
    print("case: switchnet vs cnn on plain-plasma runs", flush=True)
    train = SD.generate(hk, cfg(101, 1.0), 190, 3, start=80, states=True) + \
        SD.generate(hk, cfg(102, 1.5), 190, 3, start=80, states=True)
    held = SD.generate(hk, cfg(104, 1.0), 190, 5, start=90, states=True)
    dv = 0.2 ** 3
    x, y, e = SD.swn_nodes(train, dv)
    mean = x.mean(0); std = x.std(0); std[std <= 0] = 1.0
    swn = hk.SwitchNet(seed=5)
    swn.set_params(T.swn_init_params(3))
    losses = SD.swn_train(swn, x, y, e, mean, std, 400, B=4096, lr=1e-3)
    xh, yh, _ = SD.swn_nodes(held, dv)
    a_swn = T.auc(SD.swn_predict(swn, xh, mean, std), yh)
    cm, cs = SD.stats(train)
    cnn = hk.CNN(seed=5)
    cnn.set_params(T.init_params(3))
    SD.train(cnn, train, cm, cs, 400, B=8, lr=1e-3, dv=dv)
    a_cnn = T.auc(np.concatenate([SD.predict(cnn, d[0], cm, cs).ravel() for d in held]), yh)
    a_now = T.auc(np.concatenate([d[3].ravel() for d in held]), yh)
    print("SwitchNet loss first %.3f last 50 %.3f; held-out AUC: SwitchNet %.4f, CNN %.4f, threshold now %.4f" % (
        losses[0], np.mean(losses[-50:]), a_swn, a_cnn, a_now))
    assert np.mean(losses[-50:]) < losses[0]
    assert a_swn > 0.6
