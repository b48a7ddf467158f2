"""Training data and training loop of the next-state surrogate, on the GPU.

Paper: Results, the StatePredictor paragraph and Table 2 (a residual 3D CNN
learns the state of a 16^3 patch a few steps ahead from the present one,
trained on simulation data with a Huber loss and a penalty on field-energy
violation).  The simulation makes the states in the library (hk_node_state)
and the network trains with its own BF16 matrix-core kernels and AdamW
(hk_sp_train_step).  This module only pairs snapshots, fixes the statistics
and cuts patches.
"""
from __future__ import annotations

import copy

PATCH = 16


def collect(hk, cfg, steps, every, horizon, start=0, precision="f32", mode="all_pic"):
    """Run `cfg` for start + steps + horizon steps; from step `start`, every
    `every` steps, pair the node state with the one `horizon` steps later.
    Returns a list of (state_t, state_t+horizon), torch [nz, ny, NX, 10]."""
    c = copy.deepcopy(cfg)
    c["run"]["switch_mode"] = mode
    sim = hk.Sim(c, precision=precision)
    snaps = {}
    for s in range(start + steps + horizon + 1):
        if s >= start and ((s - start) % every == 0 or (s - start - horizon) % every == 0):
            snaps[s] = sim.node_state().clone()
        sim.step(1)
    sim.close()
    return [(snaps[s], snaps[s + horizon]) for s in range(start, start + steps + 1, every) if s + horizon in snaps]


def stats(pairs):
    """Per-channel mean and standard deviation over every snapshot (float32
    numpy arrays of 10); a channel that never varies gets std 1."""
    import torch
    x = torch.stack([a for a, _ in pairs] + [b for _, b in pairs]).reshape(-1, 10).double()
    mean = x.mean(0)
    std = x.std(0)
    std = torch.where(std > 0, std, torch.ones_like(std))
    return mean.float().cpu().numpy(), std.float().cpu().numpy()


def patches(pairs, mean, std, B, gen, size=PATCH):
    """B random size^3 crops (x, y) of normalized states, [B, size, size, size, 10]."""
    import torch
    m = torch.tensor(mean, device="cuda")
    s = torch.tensor(std, device="cuda")
    xs, ys = [], []
    nz, ny, nx, _ = pairs[0][0].shape
    for _ in range(B):
        i = int(torch.randint(len(pairs), (1,), generator=gen))
        z0 = int(torch.randint(nz - size + 1, (1,), generator=gen))
        y0 = int(torch.randint(ny - size + 1, (1,), generator=gen))
        x0 = int(torch.randint(nx - size + 1, (1,), generator=gen))
        a, b = pairs[i]
        xs.append(a[z0:z0 + size, y0:y0 + size, x0:x0 + size])
        ys.append(b[z0:z0 + size, y0:y0 + size, x0:x0 + size])
    x = (torch.stack(xs) - m) / s
    y = (torch.stack(ys) - m) / s
    return x.contiguous(), y.contiguous()


def train(sp, pairs, mean, std, iters, B=8, lr=1e-3, delta=0.01, lam=0.1, seed=0, log=None):
    """AdamW on random patches; returns the losses."""
    import torch
    gen = torch.Generator().manual_seed(seed)
    sp.set_norm(mean, std)
    losses = []
    for it in range(iters):
        x, y = patches(pairs, mean, std, B, gen)
        losses.append(sp.train_step(x, y, lr=lr, delta=delta, lam=lam, dropout=True))
        if log and it % 20 == 0:
            log("iter %d loss %.5f" % (it, losses[-1]))
    return losses


def r2(sp, x, y):
    """Coefficient of determination of the prediction over all voxels and
    channels of normalized patches (the paper reports it for the surrogate)."""
    p = sp.forward(x)
    ss_res = float(((p - y) ** 2).sum())
    ss_tot = float(((y - y.mean()) ** 2).sum())
    return 1.0 - ss_res / ss_tot
