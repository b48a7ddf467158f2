"""The learned switch's training on the GPU: marshalling around the library.

Paper: Methodology, pipeline paragraph (the regime classifier is trained on
data the simulations generate, with uncertainty from Monte Carlo dropout and
a physics penalty on energy violation).  Everything numeric runs in the
library: all-PIC runs fill a device training set with node inputs, labels
and conversion energies (hk_dump_training), its per-channel statistics are
reduced on the device (hk_dataset_stats), and the network is trained on
crops sampled, normalized and weighted on the device by its own BF16
matrix-core forward and backward kernels and AdamW (hk_train).  This module
picks runs and passes arguments, plus the initial parameters and the AUC
used to score predictions.
"""
from __future__ import annotations

import copy

import numpy as np


def node_dims(cfg):
    g = cfg["grid"]
    nx = g["nx"] if g.get("bc_x", "open") == "periodic" else g["nx"] + 1
    return g["nz"], g["ny"], nx


def init_params(seed=0):
    """He-normal convolution weights, zero biases, small head (FP32 vector in the
    library's parameter layout)."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin in (8, 32, 32, 32):
        parts.append(rng.normal(0, np.sqrt(2.0 / (27 * cin)), 27 * cin * 32))
        parts.append(np.zeros(32))
    parts.append(rng.normal(0, np.sqrt(1.0 / 32), 32))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def sp_init_params(seed=0):
    """Next-state surrogate: He-normal convolution weights and zero biases in
    the library's parameter layout (per layer W[27][cin][cout], b[cout])."""
    rng = np.random.default_rng(seed)
    parts = []
    for cin, cout in zip((10, 13, 32, 64, 128, 32), (13, 32, 64, 128, 32, 10)):
        parts.append(rng.normal(0, np.sqrt(2.0 / (27 * cin)), 27 * cin * cout))
        parts.append(np.zeros(cout))
    return np.concatenate(parts).astype(np.float32)


def swn_init_params(seed=0):
    """SwitchNet: He-normal weights (W[in][out]) and zero biases in the
    library's parameter layout; a small head."""
    rng = np.random.default_rng(seed)
    parts = []
    for ni, no in [(10, 128), (128, 256)] + [(256, 256)] * 4:
        parts.append(rng.normal(0, np.sqrt(2.0 / ni), ni * no))
        parts.append(np.zeros(no))
    parts.append(rng.normal(0, np.sqrt(1.0 / 256), 256))
    parts.append(np.zeros(1))
    return np.concatenate(parts).astype(np.float32)


def build_dataset(hk, cfgs, steps, every, start=0, window=10, precision="f32", log=None):
    """A device training set from all-PIC runs of each config: `start` steps
    advanced, then snapshots every `every` steps up to `steps` with labels
    over the next `window` steps (hk_dump_training)."""
    ds = hk.Dataset(precision)
    for cfg in cfgs:
        c = copy.deepcopy(cfg)
        c["run"]["switch_mode"] = "all_pic"
        sim = hk.Sim(c, precision=precision)
        if start:
            sim.step(start)
        ds.dump(sim, steps, every, window)
        sim.close()
        if log:
            log("%s: %d snapshots so far" % (c["name"], len(ds)))
    return ds


def train_switch(ds, cnn, iters, B=64, lr=1e-3, lam=0.1, seed=0):
    """Statistics of the set into the network, then hk_train; the losses."""
    mean, std = ds.stats()
    cnn.set_norm(mean, std)
    return ds.train(cnn, iters, B=B, lr=lr, lam=lam, seed=seed)


def scores(ds, cnn):
    """(network logits, threshold flags, labels) over every node of every
    snapshot, flattened: the network against the method without it."""
    ps, ts, ys = [], [], []
    for k in range(len(ds)):
        _, _, y, thr = ds.get(k)
        ps.append(ds.predict(cnn, k).cpu().numpy().ravel())
        ts.append(thr.ravel()); ys.append(y.ravel())
    return np.concatenate(ps), np.concatenate(ts), np.concatenate(ys)


def auc(score, label):
    """Area under the ROC curve (ties count half)."""
    s = np.asarray(score, float).ravel(); y = np.asarray(label).ravel() > 0.5
    npos, nneg = y.sum(), (~y).sum()
    if npos == 0 or nneg == 0:
        return float("nan")
    order = np.argsort(s, kind="mergesort")
    ranks = np.empty(len(s)); ranks[order] = np.arange(1, len(s) + 1)
    # average ranks over ties
    ss = s[order]
    i = 0
    while i < len(ss):
        j = i
        while j + 1 < len(ss) and ss[j + 1] == ss[i]:
            j += 1
        if j > i:
            ranks[order[i:j + 1]] = 0.5 * (i + j) + 1
        i = j + 1
    return float((ranks[y].sum() - npos * (npos + 1) / 2) / (npos * nneg))
