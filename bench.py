#!/usr/bin/env python
"""Benchmark of the hybrid fluid-kinetic step on one MI355X.

Workload: the full-size foil, 512 x 256 x 256 cells (33.5 M), dx = 0.05; a
pre-ionized hydrogen foil at 10 n_c, 1 lambda thick from x = 3.2, 16
particles per cell per species (132 M electrons and 132 M protons), mobile
protons, photon emission and pair creation on; a circular pulse (a0 = 5 by
default; 50 and 200 complete the sweep), waist 3 lambda, field half-width 10
centred at t = 20.  The hybrid (threshold switch re-evaluated every 10 steps,
hot particles |u| >= 0.1 kept kinetic) and all-PIC (every node kinetic) run the
same seed on the same GPU.  Each mode first advances W steps untimed (the
pulse front reaches the foil near step 300), then K steps run under the clock
(device synchronisation on both sides).  An all-PIC run with another seed
gives the field difference that sampling noise alone makes (the floor of any
comparison with one all-PIC run).

The JSON line reports the hybrid / all-PIC steps/s ratio (value), both
rates, particle pushes/s, cell-steps/s, the field relative L2 of hybrid vs
all-PIC at step W + K (and of all-PIC vs all-PIC with another seed), the
energy difference, the kinetic fractions, the push kernel's achieved HBM rate
against the roofline (algorithmic bytes over the kernel's own time from HIP
events on the library stream), the FP64 error of the FP32 step, and the FP64
CPU oracle timed on a bounded sample of the same physics.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, published
# algorithmic bytes per particle push: read cell, offsets, u, w (32 B), write
# cell, offsets, u (28 B); a QED lepton also reads and writes its FP64
# optical depth (16 B) and carries its id (8 B)
BYTES_PER_PUSH = 60
BYTES_PER_QED_PUSH = 84
BYTES_PER_TILE_CELL = 36       # E, B gather (24 B) + J flush (12 B) per cell of a kinetic tile
TILE_CELLS = 512
PUSH_SOURCES = ("paper_2510_11174_amd/csrc/k_particles.hip", "paper_2510_11174_amd/csrc/hk_pic_device.h",
                "paper_2510_11174_amd/csrc/hk_internal.h")
FLUID_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fluid_traffic_plain_256x128x128.txt")
FLUID_SOURCES = ("paper_2510_11174_amd/csrc/k_fluid.hip", "paper_2510_11174_amd/csrc/hk_internal.h")
FULL_GRID = (512, 256, 256)
HOT = 0.1                      # hot-particle threshold of the hybrid (|u|)


def traffic_file(a0):
    return os.path.join(ROOT, "profiles", "k_push_traffic_full_foil_a%g.txt" % a0)


def source_hash(files=PUSH_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path, files=PUSH_SOURCES, key="bytes_per_launch", window=None):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration)
    recorded in a profiles/ summary, or None if missing, taken on other kernel
    sources, or (window given) over another step window."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_hash") != source_hash(files):
            return None
        if window is not None and kv.get("window") != window:
            return None
        return float(kv[key])
    except (OSError, KeyError, ValueError):
        return None


def copy_calibration(mib=1024, reps=5):
    """A plain device copy of known size, for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * 1024 * 1024 // 4
    a = torch.ones(n, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_each_way": n * 4, "reps": reps}))


def workload(a0, mode, seed=None, grid=FULL_GRID):
    from paper_2510_11174_amd import configs
    cfg = configs.full_foil(a0, *grid, mode=mode, seed=seed)
    cfg["run"]["thr_hot"] = HOT
    return cfg


def run_window(cfg, warmup, steps, precision="f32", timing=True, snap=True, cnn=None):
    """W untimed steps, then K steps under the clock (device synchronisation on
    both sides); timers (HIP events on the library stream) cover the K steps.
    cnn: the switch network of a learned-switch run."""
    import numpy as np
    import torch

    from paper_2510_11174_amd import hk
    torch.cuda.empty_cache()
    torch.cuda.reset_peak_memory_stats()
    base = torch.cuda.memory_allocated()
    t0 = time.perf_counter()
    sim = hk.Sim(cfg, precision=precision)
    if cnn is not None:
        sim.set_cnn(cnn)
    torch.cuda.synchronize()
    create_s = time.perf_counter() - t0
    if warmup:
        sim.step(warmup)
    d0 = sim.diagnostics()
    sim.enable_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    seconds = time.perf_counter() - t0
    tm = sim.timers() if timing else {}
    d = sim.diagnostics()
    snaps = {c: sim.get_field(c).astype(np.float64) for c in ("ex", "ey", "ez", "bx", "by", "bz")} if snap else None
    peak_gb = (torch.cuda.max_memory_allocated() - base) / 1e9
    sim.close()
    del sim
    torch.cuda.empty_cache()
    return {"seconds": seconds, "timers": tm, "diag0": d0, "diag": d, "snaps": snaps, "create_s": create_s,
            "peak_gb": peak_gb}


def train_switch(precision="f32", iters=3200, B=64, grid=(256, 64, 64), log=None):
    """The learned switch for the foil: a device training set from all-PIC
    runs of the foil physics on a 256 x 64 x 64 box (a0 5 and 20, steps
    150-800 every 25, labels over the next 10 steps), 3200 AdamW steps on
    batches of 64 crops (204,800 crops of 24^3), scored on a held-out a0 5
    run against the threshold flags (AUC of the future kinetic label)."""
    import torch

    from paper_2510_11174_amd import configs, hk
    from paper_2510_11174_amd import train as T
    t0 = time.perf_counter()
    cfgs = [configs.full_foil(a, *grid, mode="all_pic", seed=configs.SEED_BASE + 100 + i)
            for i, a in enumerate((5.0, 20.0))]
    ds = T.build_dataset(hk, cfgs, 650, 25, start=150, precision=precision)
    held = T.build_dataset(hk, [configs.full_foil(5.0, *grid, mode="all_pic", seed=configs.SEED_BASE + 150)],
                           650, 50, start=150, precision=precision)
    t_data = time.perf_counter() - t0
    cnn = hk.CNN(seed=5, precision=precision)
    cnn.set_params(T.init_params(3))
    t0 = time.perf_counter()
    losses = T.train_switch(ds, cnn, iters, B=B, lr=1e-3)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t0
    p, thr, y = T.scores(held, cnn)
    info = {"snapshots": len(ds), "crops": iters * B, "data_s": round(t_data, 1), "train_s": round(t_train, 1),
            "loss_first": float(sum(losses[:20]) / 20), "loss_last": float(sum(losses[-100:]) / 100),
            "heldout_auc_network": round(T.auc(p, y), 4), "heldout_auc_threshold": round(T.auc(thr, y), 4),
            "heldout_label_fraction": round(float(y.mean()), 4),
            "data": "all-PIC foil physics 256x64x64, a0 5 and 20, steps 150-800 every 25; held-out a0 5 run"}
    ds.close(); held.close()
    return cnn, info


def total_energy(d):
    return (d["u_e"] + d["u_b"] + sum(d["kin"]) + sum(d["fluid_kin"]) + sum(d["fluid_th"]) + d["conv_loss"]
            + d["ion_energy"] + d["photon_energy"])


def field_l2(x, y):
    import numpy as np
    num = math.sqrt(sum(float(np.sum((x[c] - y[c]) ** 2)) for c in x))
    den = math.sqrt(sum(float(np.sum(y[c] ** 2)) for c in y))
    return num / den if den > 0 else 0.0


def push_roofline(r, kind_bytes):
    """k_push over the timed window: algorithmic bytes (per species: particles
    in the window's diagnostics times the steps, 84 B for a QED lepton, 60 B
    otherwise, plus 36 B per cell of every tile pushed) over the push's own
    time (HIP events on the library stream)."""
    tm = r["timers"]
    ms = tm["push_kernel_ms"]
    launches = max(tm["push_launches"], 1)
    alg = kind_bytes * 1.0 + BYTES_PER_TILE_CELL * TILE_CELLS * tm["tiles_pushed"]
    achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
    return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": round(achieved / HBM_PEAK_GBS, 4), "kernel": "k_push", "avg_launch_ms": round(ms / launches, 4),
            "launches": int(launches), "alg_bytes_per_launch": round(alg / launches)}


def particle_bytes(cfg, r, steps):
    """Algorithmic push bytes of a window: each species' count (mean of the
    window's first and last diagnostics) times steps times its bytes per push."""
    tot = 0.0
    for i, sp in enumerate(cfg["species"]):
        n = 0.5 * (r["diag0"]["count"][i] + r["diag"]["count"][i])
        qed = sp.get("qed") and sp["kind"] in ("electron", "positron")
        if sp["kind"] == "photon":
            continue
        tot += n * steps * (BYTES_PER_QED_PUSH if qed else BYTES_PER_PUSH)
    return tot


def fp64_error(steps=200):
    """FP64 error of the FP32 step on a crop of the foil physics: the FP32 and
    FP64 builds run the same 128 x 64 x 64 hybrid (foil from x = 1.6, a0 = 5,
    pulse centred at t = 4) for `steps` steps; the field relative L2 between
    them, the relative total-energy difference and the kinetic fractions."""
    import numpy as np

    from paper_2510_11174_amd import configs, hk
    cfg = configs.full_foil(5.0, 128, 64, 64, mode="threshold")
    cfg["run"]["thr_hot"] = HOT
    for sp in cfg["species"]:
        if sp.get("profile") == "foil":
            sp["x0"] = 1.6
    cfg["laser"]["t_center"] = 4.0
    out = {}
    for prec in ("f32", "f64"):
        sim = hk.Sim(cfg, precision=prec)
        sim.step(steps)
        out[prec] = ({c: sim.get_field(c).astype(np.float64) for c in ("ex", "ey", "ez", "bx", "by", "bz")},
                     sim.diagnostics())
        sim.close()
    f32, f64 = out["f32"], out["f64"]
    e32, e64 = total_energy(f32[1]), total_energy(f64[1])
    return {"field_rel_l2_f32_vs_f64": field_l2(f32[0], f64[0]),
            "energy_rel_diff_f32_vs_f64": abs(e32 - e64) / abs(e64) if e64 else 0.0,
            "kinetic_fraction_f32": f32[1]["kinetic_fraction"], "kinetic_fraction_f64": f64[1]["kinetic_fraction"],
            "workload": "hybrid foil crop 128x64x64 (foil from x = 1.6, a0 5, pulse centre t = 4), %d steps" % steps}


def _oracle_rate(args):
    """One oracle process: the crop of the foil physics, `steps` timed steps."""
    nx, ny, nz, steps, warm, mode = args
    import oracle
    from paper_2510_11174_amd import configs
    cfg = configs.full_foil(5.0, nx, ny, nz, mode=mode)
    cfg["run"]["thr_hot"] = HOT
    for sp in cfg["species"]:
        if sp.get("profile") == "foil":
            sp["x0"] = 1.6
    cfg["laser"]["t_center"] = 4.0
    o = oracle.Oracle(cfg)
    o.step(warm)
    n = sum(o.count(i) for i in range(len(cfg["species"])))
    t0 = time.perf_counter()
    o.step(steps)
    dt = time.perf_counter() - t0
    return steps / dt, n * steps / dt


def cpu_baseline(steps=4, warm=1, crop=(64, 32, 32)):
    """The FP64 oracle (plain C loops, as it stands) on a crop of the foil
    physics (64 x 32 x 32 cells, foil from x = 1.6, hybrid threshold switch):
    one process on one core, and one process per host core at once (independent
    crops: the rate a domain decomposition over every core would reach at
    best).  Steps/s are scaled to the full 512 x 256 x 256 grid by the cell
    ratio."""
    import multiprocessing as mp
    import platform
    import oracle
    oracle.build(force=False)
    nx, ny, nz = crop
    scale = (nx * ny * nz) / float(FULL_GRID[0] * FULL_GRID[1] * FULL_GRID[2])
    t0 = time.perf_counter()
    one = _oracle_rate((nx, ny, nz, steps, warm, "threshold"))
    t_one = time.perf_counter() - t0
    cores = min(os.cpu_count() or 1, 16)
    ctx = mp.get_context("spawn")
    t0 = time.perf_counter()
    with ctx.Pool(cores) as pool:
        many = pool.map(_oracle_rate, [(nx, ny, nz, steps, warm, "threshold")] * cores)
    t_many = time.perf_counter() - t0
    agg_sps = sum(r[0] for r in many)
    agg_pps = sum(r[1] for r in many)
    model = ""
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"value": round(agg_sps * scale, 6), "unit": "steps/s", "cores": cores, "kind": "oracle",
            "sample": "FP64 oracle, hybrid threshold switch on a %dx%dx%d crop of the foil physics (foil from "
                      "x = 1.6, a0 5, pulse centre t = 4), steps %d-%d, one process per core on %d cores "
                      "(%.1f s); steps/s scaled to the 512x256x256 grid by the cell ratio %.0f" % (
                          nx, ny, nz, warm, warm + steps, cores, t_many, 1 / scale),
            "pushes_per_s": round(agg_pps, 1),
            "one_core": {"steps_per_s_scaled": round(one[0] * scale, 8), "pushes_per_s": round(one[1], 1),
                         "seconds": round(t_one, 1)},
            "host": {"nproc": os.cpu_count(), "cpu": model, "machine": platform.machine()}}


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16


def cnn_inference(reps=20):
    """One learned-switch evaluation's network pass on the ionizing-helium node
    grid (129 x 64 x 64 nodes with the 4-node halo), timed with HIP events on
    the library stream.  Algorithmic flops are those of the nodes the switch
    decides: 179,776 per node for the four convolutions and the head (the
    halo's partial layers are overhead, not counted)."""
    import torch

    from paper_2510_11174_amd import hk
    from paper_2510_11174_amd import train as T
    D, H, W = 64 + 8, 64 + 8, 129 + 8
    cnn = hk.CNN(seed=1)
    cnn.set_params(T.init_params(1))
    x = torch.randn((1, D, H, W, 8), device="cuda", dtype=torch.float32)
    per_node = 2 * 27 * (8 * 32 + 3 * 32 * 32) + 2 * 32
    nodes = (D - 8) * (H - 8) * (W - 8)
    flops = per_node * nodes
    cnn.forward(x)
    torch.cuda.synchronize()
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    a.record()
    for _ in range(reps):
        cnn.forward(x)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    cnn.close()
    tf = flops / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "kernel": "k_conv_fwd_first + 3 x k_conv_fwd_rows + k_head",
            "ms_per_eval": round(ms, 3), "flop_per_node": per_node, "nodes": nodes, "flop_per_eval": flops,
            "grid": "129 x 64 x 64 nodes (+ halo 4)"}


SP_CIN, SP_COUT = (10, 13, 32, 64, 128, 32), (13, 32, 64, 128, 32, 10)


def sp_surrogate(B=64, reps=20, train_reps=5):
    """The next-state surrogate on B patches of 16^3 nodes (the paper's grid
    size): one forward pass and one training step (forward, loss, both
    gradients, AdamW), timed with HIP events on the library stream.  Flops are
    those of the six convolutions with their real channel counts: forward
    2 * 27 * sum(cin cout) per voxel, training three times that less the data
    gradient of the first layer, which is not needed."""
    import torch

    from paper_2510_11174_amd import hk
    from paper_2510_11174_amd import train as T
    sp = hk.StatePredictor(seed=1)
    sp.set_params(T.sp_init_params(1))
    x = torch.randn((B, 16, 16, 16, 10), device="cuda", dtype=torch.float32)
    y = 0.9 * x
    out = torch.empty_like(x)
    nvox = B * 16 ** 3
    f = [2 * 27 * ci * co * nvox for ci, co in zip(SP_CIN, SP_COUT)]
    flops_fwd, flops_train = sum(f), 3 * sum(f) - f[0]
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        sp.forward(x, out=out)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        sp.forward(x, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    sp.train_step(x, y, lr=1e-5)
    torch.cuda.synchronize()
    a.record()
    for _ in range(train_reps):
        sp.train_step(x, y, lr=1e-5)
    b.record()
    torch.cuda.synchronize()
    ms_t = a.elapsed_time(b) / train_reps
    sp.close()
    tf = flops_fwd / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "kernel": "k_sp_conv (6 layers, forward)",
            "ms_forward": round(ms, 3), "flop_forward": flops_fwd, "ms_train_step": round(ms_t, 3),
            "train_tflops": round(flops_train / (ms_t * 1e-3) / 1e12, 1), "patches": "%d x 16^3" % B}


def swn_inference(reps=20, train_nodes=65536, train_reps=5):
    """The paper's SwitchNet over every node of the ionizing-helium grid (129 x
    64 x 64 nodes), timed with HIP events on the library stream, and one
    training step on a batch of 65536 nodes.  Flops per node are those the
    method needs: the two linear blocks, the attention's value and output
    projections (a single-token softmax is 1, so the query and key
    projections do not change the result) and the head,
    2 (10*128 + 128*256 + 2*256*256 + 256)."""
    import torch

    from paper_2510_11174_amd import hk
    from paper_2510_11174_amd import train as T
    n = 129 * 64 * 64
    swn = hk.SwitchNet(seed=1)
    swn.set_params(T.swn_init_params(1))
    x = torch.randn((n, 10), device="cuda", dtype=torch.float32)
    out = torch.empty(n, device="cuda", dtype=torch.float32)
    fpn = 2 * (10 * 128 + 128 * 256 + 2 * 256 * 256 + 256)
    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    for _ in range(3):
        swn.forward(x, out=out)
    torch.cuda.synchronize()
    a.record()
    for _ in range(reps):
        swn.forward(x, out=out)
    b.record()
    torch.cuda.synchronize()
    ms = a.elapsed_time(b) / reps
    xt = x[:train_nodes].contiguous()
    y = (xt[:, 0] > 0).float()
    e = torch.ones(train_nodes, device="cuda")
    swn.train_step(xt, y, e, lr=1e-5)
    torch.cuda.synchronize()
    a.record()
    for _ in range(train_reps):
        swn.train_step(xt, y, e, lr=1e-5)
    b.record()
    torch.cuda.synchronize()
    ms_t = a.elapsed_time(b) / train_reps
    swn.close()
    tf = fpn * n / (ms * 1e-3) / 1e12
    return {"bound": "mfma", "achieved": round(tf, 1), "peak": MFMA_BF16_PEAK_TFLOPS, "unit": "TFLOP/s",
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "kernel": "k_sp_conv one-tap (5 linear layers)",
            "ms_forward": round(ms, 3), "flop_per_node": fpn, "nodes": n,
            "ms_train_step": round(ms_t, 3), "train_nodes": train_nodes}


def laser_search(pop=8, gens=3, steps=120):
    """The laser-parameter search (differential evolution over a0, duration and
    waist) on the underdense 32x16x16 plasma: pop * (gens + 1) hybrid runs of
    `steps` steps each, FP32 library, timed on the host clock."""
    from paper_2510_11174_amd import configs, hk, optimize
    cfg = configs.plain_hybrid(32, 16, 16)
    target = optimize.run_energy(hk, cfg, [1.2, 3.5, 6.0], steps)
    r = optimize.optimize_laser(hk, cfg, target, [0.5, 2.0, 2.0], [2.0, 5.0, 10.0], steps, pop=pop, gens=gens,
                                seed=3)
    return {"runs": r["evaluations"], "steps_per_run": steps, "seconds": round(r["seconds"], 3),
            "runs_per_s": round(r["runs_per_s"], 2), "hybrid_steps_per_s": round(r["steps_per_s"], 1),
            "rel_error": r["rel_error"], "workload": "plain_hybrid_32x16x16, DE pop %d, %d generations" % (pop, gens)}


def warm_fluid(steps=200, warmup=20, nx=256, ny=128, nz=128):
    """The fluid phase of the step on an all-fluid plasma (the underdense case
    at 256 x 128 x 128 cells, electrons at u_th 0.05 absorbed into the node
    fluid at the first step, then laser and fluid only), warm (adiabatic,
    gamma 5/3) and cold.  Time: the library's HIP events around the fluid
    passes on its stream, over `steps` steps after `warmup`.  Algorithmic
    bytes per node and step: read n, u (4), E, B (6), J (3) and write n, u (4):
    17 values, 68 B in FP32; a warm fluid also reads and writes S (76 B)."""
    from paper_2510_11174_amd import configs, hk
    out = {}
    nodes = (nx + 1) * ny * nz
    for name, ga in (("warm", 5.0 / 3.0), ("cold", 0.0)):
        cfg = configs.plain_hybrid(nx, ny, nz, mode="all_fluid")
        cfg["species"][0]["u_th"] = 0.05
        cfg["species"][0]["gamma_ad"] = ga
        sim = hk.Sim(cfg, precision="f32")
        sim.step(1 + warmup)
        sim.enable_timing(True)
        t0 = time.perf_counter()
        sim.step(steps)
        import torch
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        tm = sim.timers()
        d = sim.diagnostics()
        sim.close()
        ms = tm["fluid_ms"] / steps
        alg = (19 if ga > 0 else 17) * 4 * nodes
        gbs = alg / (ms * 1e-3) / 1e9
        out[name] = {"ms_fluid_per_step": round(ms, 4), "alg_bytes_per_step": alg,
                     "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "steps_per_s": round(steps / sec, 1), "fluid_heat": d["fluid_th"][0]}
    c = out["cold"]
    traffic = measured_traffic(FLUID_TRAFFIC_FILE, FLUID_SOURCES, "bytes_per_step_cold")
    return {"bound": "hbm", "achieved": c["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": c["frac"],
            "traffic": traffic, "kernel": "k_fluid_lorentz + k_fluid_update (cold)", "nodes": nodes,
            "workload": "plain plasma %dx%dx%d, all fluid, u_th 0.05" % (nx, ny, nz), **{k: v for k, v in out.items()}}


def _csv_rows(d, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))
    if not files:
        print("no *%s under %s" % (suffix, d), file=sys.stderr)
        sys.exit(1)
    with open(files[0], newline="") as fh:
        return list(csv.DictReader(fh))


def _short_name(name):
    """A kernel's name without return type and namespace: 'void
    (anonymous namespace)::k_push<1>(GridP, ...)' gives 'k_push<1>'."""
    n = name
    if n.startswith("void "):
        n = n[5:]
    n = n.replace("(anonymous namespace)::", "")
    return n.split("(", 1)[0]


def _is_kernel(name, kernel):
    """Whether the dispatch `name` is `kernel` (any template instance)."""
    n = _short_name(name)
    return n == kernel or n.startswith(kernel + "<")


def summarize_trace(d, kernel, last):
    """Kernel-time summary of a rocprofv3 --kernel-trace --stats --output-format
    csv directory: the mean duration of the last `last` dispatches of
    `kernel` (the timed window), then the per-kernel table of the whole run."""
    rows = [r for r in _csv_rows(d, "kernel_trace.csv") if _is_kernel(r["Kernel_Name"], kernel)]
    rows.sort(key=lambda r: int(r["Start_Timestamp"]))
    sel = rows[-last:] if last else rows
    dur = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) * 1e-3 for r in sel]
    print("%s: %d dispatches in the run; the last %d: mean %.1f us, min %.1f, max %.1f" % (
        kernel, len(rows), len(sel), sum(dur) / max(len(dur), 1), min(dur), max(dur)))
    stats = _csv_rows(d, "kernel_stats.csv")
    tot = sum(float(r["TotalDurationNs"]) for r in stats)
    print("\nAll kernels of the run (kernel_stats.csv):")
    print("%-44s %8s %11s %9s %7s" % ("kernel", "calls", "total ms", "avg us", "%"))
    for r in sorted(stats, key=lambda r: -float(r["TotalDurationNs"]))[:28]:
        print("%-44s %8s %11.2f %9.1f %7.2f" % (_short_name(r["Name"])[:44], r["Calls"],
                                                float(r["TotalDurationNs"]) * 1e-6,
                                                float(r["AverageNs"]) * 1e-3,
                                                100.0 * float(r["TotalDurationNs"]) / tot))


def _counter_per_dispatch(d, kernel=None, name_re=None):
    import re
    per = {}
    for r in _csv_rows(d, "counter_collection.csv"):
        n = r["Kernel_Name"]
        if kernel and not _is_kernel(n, kernel):
            continue
        if name_re and not re.search(name_re, n, re.I):
            continue
        key = int(r["Dispatch_Id"])
        per[key] = per.get(key, 0.0) + float(r["Counter_Value"])
    return [per[k] for k in sorted(per)]


def summarize_counters(d, kernel, last):
    """Mean per dispatch of every counter in a rocprofv3 --pmc csv directory,
    for each instance of `kernel` (template arguments apart), over the last
    `last` dispatches of the kernel (all when 0)."""
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True))
    if not files:
        print("no counter_collection.csv under %s" % d, file=sys.stderr)
        sys.exit(1)
    per, name, info = {}, {}, {}
    with open(files[0], newline="") as fh:
        for r in csv.DictReader(fh):
            if not _is_kernel(r["Kernel_Name"], kernel):
                continue
            did = int(r["Dispatch_Id"])
            per.setdefault(did, {})
            per[did][r["Counter_Name"]] = per[did].get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
            name[did] = _short_name(r["Kernel_Name"])
            info[name[did]] = (r.get("Workgroup_Size"), r.get("LDS_Block_Size"), r.get("VGPR_Count"),
                               r.get("SGPR_Count"))
    ids = sorted(per)[-last:] if last else sorted(per)
    for inst in sorted(set(name[i] for i in ids)):
        sel = [i for i in ids if name[i] == inst]
        keys = sorted(set(k for i in sel for k in per[i]))
        wg, lds, vgpr, sgpr = info[inst]
        print("%s: %d dispatches (workgroup %s, LDS %s B, VGPR field %s, SGPR %s)" % (inst, len(sel), wg, lds,
                                                                                     vgpr, sgpr))
        for k in keys:
            print("  %-32s %.6g" % (k, sum(per[i].get(k, 0.0) for i in sel) / len(sel)))


def summarize_traffic(a):
    """HBM traffic of `kernel` per dispatch from two rocprofv3 --pmc csv runs
    (FETCH_SIZE, WRITE_SIZE; KiB per dispatch, the last `last` dispatches)
    scaled by what the same counters read for a 1 GiB device copy (two more
    runs of bench.py --calibrate-copy).  Prints a profiles/ summary body."""
    known = 1024 ** 3
    cf = [v for v in _counter_per_dispatch(a.calib_fetch, name_re="copy") if v * 1024 > known / 8]
    cw = [v for v in _counter_per_dispatch(a.calib_write, name_re="copy") if v * 1024 > known / 8]
    f_scale = known / (1024 * sum(cf) / len(cf))
    w_scale = known / (1024 * sum(cw) / len(cw))
    f = _counter_per_dispatch(a.fetch, kernel=a.kernel)
    w = _counter_per_dispatch(a.write, kernel=a.kernel)
    f, w = f[-a.last:], w[-a.last:]
    fk, wk = sum(f) / len(f), sum(w) / len(w)
    fb, wb = fk * 1024 * f_scale, wk * 1024 * w_scale
    print("# Calibration: a 1 GiB device copy reads FETCH_SIZE %.0f KiB and WRITE_SIZE %.0f KiB," % (
        sum(cf) / len(cf), sum(cw) / len(cw)))
    print("# so FETCH_SIZE is scaled by %.4f and WRITE_SIZE by %.4f to bytes." % (f_scale, w_scale))
    print("# %s dispatches averaged: %d (FETCH), %d (WRITE)" % (a.kernel, len(f), len(w)))
    print("fetch_kib_per_launch = %.1f" % fk)
    print("write_kib_per_launch = %.1f" % wk)
    print("fetch_bytes_per_launch = %.0f" % fb)
    print("write_bytes_per_launch = %.0f" % wb)
    print("bytes_per_launch = %.0f" % (fb + wb))
    if a.alg_bytes:
        print("algorithmic_bytes_per_launch = %.0f" % a.alg_bytes)
        print("traffic_over_algorithmic = %.3f" % ((fb + wb) / a.alg_bytes))
    if a.window:
        print("window = %s" % a.window)
    print("source_hash = %s" % source_hash())
    print("# source_hash: sha256 (first 16 hex) of %s" % ", ".join(PUSH_SOURCES))


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500, help="timed steps per mode (K)")
    ap.add_argument("--warmup", type=int, default=300, help="untimed steps before the clock (W)")
    ap.add_argument("--a0", type=float, default=5.0, help="pulse amplitude of the foil workload")
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the workload's modes (no seed floor, networks, fluid, search, FP64 check)")
    ap.add_argument("--modes", default="cnn,threshold,all_pic",
                    help="comma list of switch modes to run: cnn (trains the switch network first), threshold, "
                         "all_pic (profiling runs may pick one)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--warm-fluid-only", action="store_true",
                    help="only measure the fluid phase (warm and cold) on the all-fluid 256x128x128 plasma")
    ap.add_argument("--networks-only", action="store_true",
                    help="only measure the switch CNN, the next-state surrogate and SwitchNet and print their JSON")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="print the kernel-time summary of a rocprofv3 --kernel-trace --stats csv DIR")
    ap.add_argument("--summarize-counters", metavar="DIR",
                    help="print per-dispatch counter means of --kernel from a rocprofv3 --pmc csv DIR")
    ap.add_argument("--summarize-traffic", action="store_true",
                    help="print the HBM traffic summary from --fetch/--write/--calib-fetch/--calib-write DIRs")
    ap.add_argument("--fetch"); ap.add_argument("--write")
    ap.add_argument("--calib-fetch"); ap.add_argument("--calib-write")
    ap.add_argument("--alg-bytes", type=float, default=0.0, help="algorithmic bytes per launch")
    ap.add_argument("--window", default="", help="step window the counters cover")
    ap.add_argument("--last", type=int, default=0, help="summarize the last N dispatches of --kernel")
    ap.add_argument("--kernel", default="k_push")
    args = ap.parse_args()
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.kernel, args.last)
        return
    if args.summarize_traffic:
        summarize_traffic(args)
        return
    if args.summarize_counters:
        summarize_counters(args.summarize_counters, args.kernel, args.last)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path (domain decomposition) is not "
              "implemented by this library; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    if args.networks_only:
        print(json.dumps({"roofline_cnn_switch": cnn_inference(), "roofline_state_predictor": sp_surrogate(),
                          "roofline_switchnet": swn_inference()}))
        return
    if args.calibrate_copy:
        copy_calibration()
        return
    if args.warm_fluid_only:
        print(json.dumps({"roofline_warm_fluid": warm_fluid()}))
        return

    W, K, a0 = args.warmup, args.steps, args.a0
    modes = [m for m in args.modes.split(",") if m]
    if any(m not in ("cnn", "threshold", "all_pic") for m in modes) or not modes:
        print("--modes takes cnn, threshold and/or all_pic", file=sys.stderr)
        sys.exit(2)
    window = "a0 %g, steps %d-%d" % (a0, W, W + K)
    res, cfgs = {}, {}
    net, net_info = None, None
    if "cnn" in modes:
        print("bench: training the switch network on foil-physics crops", file=sys.stderr, flush=True)
        net, net_info = train_switch(args.precision)
        print("bench: network trained (%s)" % net_info, file=sys.stderr, flush=True)
    floor_snaps = None
    if not args.no_extras and "all_pic" in modes and len(modes) >= 2:
        # all-PIC with another seed, run first so that the all-PIC window below
        # is the last stretch of push launches in the process: the field
        # difference sampling noise alone makes against one all-PIC run
        seed2 = workload(a0, "all_pic")["run"]["seed"] + 7919
        print("bench: all-PIC with seed %#x (sampling floor), steps 0-%d untimed" % (seed2, W + K),
              file=sys.stderr, flush=True)
        floor_snaps = run_window(workload(a0, "all_pic", seed=seed2), W, K, args.precision, timing=False)["snaps"]
    for mode in sorted(modes, key=lambda m: m == "all_pic"):
        cfg = workload(a0, mode)
        cfgs[mode] = cfg
        print("bench: %s %s: steps 0-%d untimed, %d-%d timed" % (cfg["name"], mode, W, W, W + K),
              file=sys.stderr, flush=True)
        res[mode] = run_window(cfg, W, K, args.precision, cnn=net if mode == "cnn" else None)
        print("bench: %s %.3f ms/step" % (mode, 1e3 * res[mode]["seconds"] / K), file=sys.stderr, flush=True)
    if "all_pic" not in res or len(res) < 2:
        mode = modes[0]
        r = res[mode]
        print(json.dumps({"mode": mode, "steps_per_s": K / r["seconds"], "window": window,
                          "roofline": push_roofline(r, particle_bytes(cfgs[mode], r, K)),
                          "timers": r["timers"], "kinetic_fraction": r["diag"]["kinetic_fraction"],
                          "count": r["diag"]["count"]}))
        return
    p = res["all_pic"]
    floor = field_l2(floor_snaps, p["snaps"]) if floor_snaps is not None else None
    pic_sps = K / p["seconds"]
    e_p = total_energy(p["diag"])
    parts_p = sum(p["diag"]["count"][:2]) + sum(p["diag0"]["count"][:2])
    cells = FULL_GRID[0] * FULL_GRID[1] * FULL_GRID[2]

    def hybrid_entry(mode):
        h = res[mode]
        sps = K / h["seconds"]
        l2 = field_l2(h["snaps"], p["snaps"])
        drift = abs(total_energy(h["diag"]) - e_p) / abs(e_p) if e_p else 0.0
        parts = sum(h["diag"]["count"][:2]) + sum(h["diag0"]["count"][:2])
        roof_h = push_roofline(h, particle_bytes(cfgs[mode], h, K))
        roof_h["traffic"] = None
        return {"switch": mode, "steps_per_s": round(sps, 2), "ratio_vs_allpic": round(sps / pic_sps, 3),
                "ms_per_step": round(1e3 / sps, 4),
                "pushes_per_s": round(h["timers"]["particles_pushed"] / h["seconds"], 1),
                "cell_steps_per_s": round(cells * sps, 1),
                "field_rel_l2_vs_allpic": l2, "energy_diff_vs_allpic": drift,
                "field_err_ok": bool(l2 <= 1e-3 and drift <= 1e-3),
                "within_pic_sampling_floor": None if floor is None else bool(l2 <= floor),
                "kinetic_fraction_nodes": h["diag"]["kinetic_fraction"],
                "fallback_fraction_nodes": h["diag"]["fallback_fraction"],
                "particle_fraction_vs_allpic": round(parts / parts_p, 4) if parts_p else None,
                "roofline_push": roof_h,
                "timers_ms_per_step": {k: round(v / K, 4) for k, v in h["timers"].items() if k.endswith("_ms")},
                "rebins": h["timers"]["rebins"], "create_s": round(h["create_s"], 2),
                "device_memory_peak_gb": round(h["peak_gb"], 1)}

    hyb = {m: hybrid_entry(m) for m in ("cnn", "threshold") if m in res}
    head = hyb["cnn"] if "cnn" in hyb else hyb["threshold"]
    traffic = measured_traffic(traffic_file(a0), window=window)
    roof = push_roofline(p, particle_bytes(cfgs["all_pic"], p, K))
    roof["traffic"] = traffic
    sw = "learned (CNN with threshold fallback)" if head["switch"] == "cnn" else "threshold"
    out = {
        "metric": "hybrid steps/s vs all-PIC on same GPU at field err <=1e-3; particle pushes/s",
        "value": head["ratio_vs_allpic"],
        "unit": "x (hybrid / all-PIC steps/s)",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": "full-size learned-hybrid workload, foil target: 512x256x256 cells, dx 0.05, "
                               "H foil 10 n_c 1 lambda thick, 16 ppc per species, QED on, CP a0 %g; %s switch "
                               "every 10 steps (hot |u| >= %g kinetic) vs all-PIC, same seed; steps %d-%d timed "
                               "after %d untimed" % (a0, sw, HOT, W, W + K, W),
                   "grid": list(FULL_GRID), "ppc": 16, "a0": a0, "switch": head["switch"], "switch_every": 10},
        "hybrid_steps_per_s": head["steps_per_s"],
        "allpic_steps_per_s": round(pic_sps, 2),
        "pushes_per_s": head["pushes_per_s"],
        "allpic_pushes_per_s": round(p["timers"]["particles_pushed"] / p["seconds"], 1),
        "cell_steps_per_s": head["cell_steps_per_s"],
        "allpic_cell_steps_per_s": round(cells * pic_sps, 1),
        "field_rel_l2_vs_allpic": head["field_rel_l2_vs_allpic"],
        "field_rel_l2_allpic_other_seed": floor,
        "energy_diff_vs_allpic": head["energy_diff_vs_allpic"],
        "field_err_ok": head["field_err_ok"],
        "within_pic_sampling_floor": head["within_pic_sampling_floor"],
        "kinetic_fraction_nodes": head["kinetic_fraction_nodes"],
        "particle_fraction_vs_allpic": head["particle_fraction_vs_allpic"],
        "roofline": roof,
        "hybrids": hyb,
        "switch_network": net_info,
        "timers_allpic_ms_per_step": {k: round(v / K, 4) for k, v in p["timers"].items() if k.endswith("_ms")},
        "rebins_allpic": p["timers"]["rebins"],
        "create_s_allpic": round(p["create_s"], 2),
        "device_memory_peak_gb_allpic": round(p["peak_gb"], 1),
    }
    # the field update (Yee, Mur walls, antenna) of the all-PIC run, from its
    # HIP-event phase timer; algorithmic bytes per cell and step: read E, B, J
    # and write E, B once (60 B), plus the particle current's 64-bit sums read
    # once (24 B): 84 B
    f_ms = p["timers"]["fields_ms"] / K
    yee_gbs = 84 * cells / (f_ms * 1e-3) / 1e9 if f_ms > 0 else 0.0
    out["roofline_yee"] = {"bound": "hbm", "achieved": round(yee_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(yee_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                           "kernel": "k_jconvert + k_yee_step + k_antenna",
                           "ms_per_step": round(f_ms, 4), "alg_bytes_per_step": 84 * cells}
    if not args.no_extras:
        out["fp64_error"] = fp64_error()
        out["roofline_cnn_switch"] = cnn_inference()
        out["roofline_state_predictor"] = sp_surrogate()
        out["roofline_switchnet"] = swn_inference()
        out["roofline_warm_fluid"] = warm_fluid()
        out["laser_search"] = laser_search()
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
