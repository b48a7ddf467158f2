"""Host-side training data of the SwitchNet comparison (per-node labels of
the threshold criterion firing within the next steps of an all-PIC run, node
states, numpy crops for the CNN arm of that comparison).  The switch CNN of
the simulation is trained from the library's own training set
(hk_dump_training / hk_train); this module only serves the test that sets
the paper's per-node SwitchNet beside it on the labels it was built with."""
from __future__ import annotations

import copy

import numpy as np

from paper_2510_11174_amd.train import node_dims

HALO = 4
CROP = 24


def generate(hk, cfg, steps, every, start=0, window=10, precision="f32", states=False):
    """Run `cfg` all-PIC for steps + window steps; snapshots every `every`
    steps from `start`.  Returns a list of (raw[nz, ny, NX, 8], y, e, hot_now),
    with the node states [nz, ny, NX, 10] (hk_node_state) appended when
    `states` is set."""
    c = copy.deepcopy(cfg)
    c["run"]["switch_mode"] = "all_pic"
    sim = hk.Sim(c, precision=precision)
    dims = node_dims(c)
    n = int(np.prod(dims))
    hots, snaps = [], {}
    for s in range(steps + window + 1):
        raw, e, hot = sim.node_inputs()
        hots.append(hot.reshape(dims))
        if s >= start and (s - start) % every == 0 and s <= steps:
            snaps[s] = (raw, e, sim.node_state().cpu().numpy() if states else None)
        sim.step(1)
    sim.close()
    out = []
    for s, (raw, e, st) in sorted(snaps.items()):
        y = np.zeros(dims, np.float32)
        for h in hots[s:s + window + 1]:
            y = np.maximum(y, h.astype(np.float32))
        d = (raw.reshape(dims + (8,)), y, e.reshape(dims), hots[s].astype(np.float32))
        out.append(d + (st,) if states else d)
    return out


def swn_nodes(data, dv=1.0):
    """Per-node SwitchNet samples of snapshots made with states=True:
    features x[N, 10] (node states), labels y[N], energy weights e[N] (the
    conversion energy over the snapshot's mean kinetic energy per node)."""
    xs, ys, es = [], [], []
    for raw, y, e, _, st in data:
        ke = 0.5 * (raw[..., 6] * dv * raw[..., 7] ** 2).mean() + 1e-30
        xs.append(st.reshape(-1, 10)); ys.append(y.ravel()); es.append(e.ravel() / ke)
    return (np.concatenate(xs).astype(np.float32), np.concatenate(ys).astype(np.float32),
            np.concatenate(es).astype(np.float32))


def swn_train(swn, x, y, e, mean, std, iters, B=4096, lr=1e-3, lam=0.1, seed=0, log=None):
    """AdamW on random node batches (B a multiple of 8); returns the losses."""
    import torch
    rng = np.random.default_rng(seed)
    xn = torch.tensor((x - mean) / std, device="cuda")
    yd = torch.tensor(y, device="cuda"); ed = torch.tensor(e, device="cuda")
    losses = []
    for it in range(iters):
        idx = torch.tensor(rng.integers(0, len(x), B), device="cuda")
        losses.append(swn.train_step(xn[idx], yd[idx], ed[idx], lr=lr, lam=lam, dropout=True))
        if log and (it % 50 == 0 or it == iters - 1):
            log("iter %d loss %.4f" % (it, losses[-1]))
    return losses


def swn_predict(swn, x, mean, std):
    """p per node (no dropout)."""
    import torch
    xd = torch.tensor(((x - mean) / std).astype(np.float32), device="cuda")
    return torch.sigmoid(swn.forward(xd)).cpu().numpy()


def stats(data):
    x = np.concatenate([d[0].reshape(-1, 8) for d in data])
    mean = x.mean(0)
    std = x.std(0)
    std[std <= 0] = 1.0
    return mean.astype(np.float32), std.astype(np.float32)


def pad(a, periodic_x):
    """4-node halo: wrap in y and z (and periodic x), repeat the wall node in open x."""
    a = np.pad(a, [(HALO, HALO), (HALO, HALO), (0, 0)] + [(0, 0)] * (a.ndim - 3), mode="wrap")
    mode = "wrap" if periodic_x else "edge"
    return np.pad(a, [(0, 0), (0, 0), (HALO, HALO)] + [(0, 0)] * (a.ndim - 3), mode=mode)


def crops(data, mean, std, B, rng, periodic_x=False, dv=1.0):
    """B random crops: x [B, 24, 24, 24, 8] normalized, y and e [B, 16, 16, 16]."""
    xs, ys, es = [], [], []
    for _ in range(B):
        raw, y, e = data[rng.integers(len(data))][:3]
        P = pad(raw, periodic_x)
        D, H, W = y.shape
        z0 = rng.integers(0, max(1, D - 16 + 1)); y0 = rng.integers(0, max(1, H - 16 + 1))
        x0 = rng.integers(0, max(1, W - 16 + 1))
        xc = P[z0:z0 + CROP, y0:y0 + CROP, x0:x0 + CROP]
        yc = np.pad(y, [(0, 16), (0, 16), (0, 16)])[z0:z0 + 16, y0:y0 + 16, x0:x0 + 16]
        ec = np.pad(e, [(0, 16), (0, 16), (0, 16)])[z0:z0 + 16, y0:y0 + 16, x0:x0 + 16]
        if xc.shape[:3] != (CROP, CROP, CROP):
            xc = np.pad(xc, [(0, CROP - xc.shape[0]), (0, CROP - xc.shape[1]), (0, CROP - xc.shape[2]), (0, 0)],
                        mode="edge")
        # kinetic energy of the crop from the inputs: (1/2) n dV |p|_rms^2 per node
        ke = 0.5 * (raw[..., 6] * dv * raw[..., 7] ** 2).sum() + 1e-30
        xs.append((xc - mean) / std); ys.append(yc); es.append(ec / ke * yc.size)
    return (np.stack(xs).astype(np.float32), np.stack(ys).astype(np.float32),
            np.stack(es).astype(np.float32))


def train(cnn, data, mean, std, iters, B=8, lr=1e-3, lam=0.1, seed=0, periodic_x=False, dv=1.0, log=None):
    import torch
    rng = np.random.default_rng(seed)
    cnn.set_norm(mean, std)
    losses = []
    for it in range(iters):
        x, y, e = crops(data, mean, std, B, rng, periodic_x, dv)
        xd, yd, ed = (torch.tensor(a, device="cuda") for a in (x, y, e))
        losses.append(cnn.train_step(xd, yd, ed, lr=lr, lam=lam, dropout=True))
        if log and (it % 50 == 0 or it == iters - 1):
            log("iter %d loss %.4f" % (it, losses[-1]))
    return losses


def predict(cnn, raw, mean, std, periodic_x=False):
    """p over the node grid of one snapshot (no dropout)."""
    import torch
    x = (pad(raw, periodic_x) - mean) / std
    xd = torch.tensor(x[None].astype(np.float32), device="cuda")
    return torch.sigmoid(cnn.forward(xd))[0].cpu().numpy()
