"""The learned switch end to end on the GPU: training data from all-PIC runs
(hk_node_inputs), training by the library's own BF16 forward/backward kernels
and AdamW, then what the trained network gains over the method without it
(the physics threshold) on a held-out run.  The all-PIC run is the judge."""
import math

import numpy as np
import pytest

from paper_2510_11174_amd import configs
from paper_2510_11174_amd import train as T

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def hk():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2510_11174_amd import hk as hkmod
    return hkmod


def _cfg(seed, a0, mode="all_pic", every=1):
    c = configs.plain_hybrid(32, 16, 16, mode=mode, seed=seed)
    c["laser"]["a0"] = a0
    c["run"]["switch_every"] = every
    return c


def _l2(a, b):
    return math.sqrt(sum(float(((a[q] - b[q]) ** 2).sum()) for q in a)) / \
        math.sqrt(sum(float((b[q] ** 2).sum()) for q in b))


def _run(hk, cfg, cnn=None, steps=200):
    s = hk.Sim(cfg)
    if cnn is not None:
        s.set_cnn(cnn)
    kin = []
    for _ in range(steps // 10):
        s.step(10)
        kin.append(float(s.get_switch().mean()))
    f = {q: s.get_field(q).astype(np.float64) for q in ("ex", "ey", "ez", "bx", "by", "bz")}
    s.close()
    return f, float(np.mean(kin))


def test_trained_switch_gains_over_threshold(hk):
    print("case: cnn training on plain-plasma runs", flush=True)
    # training data: two seeds and laser strengths; labels = the physics
    # criterion firing within the next 10 steps of the all-PIC run
    train = T.generate(hk, _cfg(101, 1.0), 190, 3, start=80) + T.generate(hk, _cfg(102, 1.5), 190, 3, start=80)
    held = T.generate(hk, _cfg(104, 1.0), 190, 5, start=90)
    mean, std = T.stats(train)
    cnn = hk.CNN(seed=5)
    cnn.set_params(T.init_params(3))
    losses = T.train(cnn, train, mean, std, 400, B=8, lr=1e-3, dv=0.2 ** 3)
    print("loss first %.3f, last 50 %.3f" % (losses[0], np.mean(losses[-50:])))
    assert np.mean(losses[-50:]) < 0.5 * losses[0]
    # 1. where will the criterion fire in the next 10 steps? (held-out run)
    ps = np.concatenate([T.predict(cnn, d[0], mean, std).ravel() for d in held])
    ys = np.concatenate([d[1].ravel() for d in held])
    now = np.concatenate([d[3].ravel() for d in held])
    a_cnn, a_now = T.auc(ps, ys), T.auc(now, ys)
    print("AUC of the future kinetic label: network %.4f, threshold now %.4f" % (a_cnn, a_now))
    assert a_cnn > a_now + 0.1
    # 2. the hybrid with the switch evaluated every 10 steps, against all-PIC
    ref, _ = _run(hk, _cfg(104, 1.0))
    f_thr, k_thr = _run(hk, _cfg(104, 1.0, "threshold", 10))
    f_cnn, k_cnn = _run(hk, _cfg(104, 1.0, "cnn", 10), cnn=cnn)
    e_thr, e_cnn = _l2(f_thr, ref), _l2(f_cnn, ref)
    print("field L2 vs all-PIC at step 200: threshold %.3e (kinetic %.3f), network %.3e (kinetic %.3f)" % (
        e_thr, k_thr, e_cnn, k_cnn))
    assert e_cnn < e_thr
