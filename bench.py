#!/usr/bin/env python
"""Benchmark of the hybrid fluid-kinetic step on one MI355X.

Workload: the ionizing-helium case (128 x 64 x 64 cells, dx = 0.1, 8 particles
per cell, neutral He 0.1 n_c with a 10-lambda up-ramp, a0 = 10 linear pulse,
waist 6 lambda, duration 15, ADK/multiphoton ionization, threshold switch).
The same seed runs on the same GPU as hybrid (threshold switch) and as all-PIC
(every node kinetic).  Each mode first runs W untimed warm-up steps on a
throwaway simulation; then a fresh simulation runs steps 0..K from t = 0 under
the clock (device synchronisation on both sides; the field snapshot at K/2 is
taken outside the clock).  An untimed repeat of the all-PIC run measures the
run-to-run floor of the field comparison (FP32 atomics sum in varying order).

The JSON line reports hybrid steps/s (value), all-PIC steps/s, the speed-up,
particle pushes/s, the field relative L2 of hybrid vs all-PIC (and of the
all-PIC repeat) at K/2 and K, the energy difference at K, the push kernel's
achieved HBM rate against the roofline
(algorithmic bytes: 60 B per particle push plus 36 B per cell of every tile
with particles, over the kernel's own time from HIP events on the library
stream), and the FP64 CPU oracle timed on a bounded sample of the same physics.
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
BYTES_PER_PUSH = 60            # read offsets, u, w, cell (32 B); write offsets, u, cell (28 B)
BYTES_PER_TILE_CELL = 36       # E, B gather (24 B) + J flush (12 B) per cell of a kinetic tile
TILE_CELLS = 512
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_push_traffic_ionization_128x64x64.txt")
PUSH_SOURCES = ("paper_2510_11174_amd/csrc/k_particles.hip", "paper_2510_11174_amd/csrc/hk_pic_device.h",
                "paper_2510_11174_amd/csrc/hk_internal.h")
FLUID_TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_fluid_traffic_plain_256x128x128.txt")
FLUID_SOURCES = ("paper_2510_11174_amd/csrc/k_fluid.hip", "paper_2510_11174_amd/csrc/hk_internal.h")


def source_hash(files=PUSH_SOURCES):
    import hashlib
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(path=TRAFFIC_FILE, files=PUSH_SOURCES, key="bytes_per_launch"):
    """HBM bytes (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration)
    recorded in a profiles/ summary, or None if missing or taken on other kernel
    sources.  Default: per k_push launch."""
    try:
        kv = {}
        with open(path) as fh:
            for line in fh:
                if "=" in line and not line.startswith("#"):
                    k, v = line.split("=", 1)
                    kv[k.strip()] = v.strip()
        if kv.get("source_hash") != source_hash(files):
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


def run_gpu(cfg, steps, precision, timing=True, snap_at=None):
    """Run `steps` steps of a fresh simulation from t = 0.  The clock covers the
    steps only (device synchronisation on both sides of each timed segment); a
    field snapshot at step `snap_at` is taken outside the clock."""
    import numpy as np
    import torch

    from paper_2510_11174_amd import hk
    sim = hk.Sim(cfg, precision=precision)
    sim.enable_timing(timing)
    segs = [steps] if not snap_at else [snap_at, steps - snap_at]
    seconds = 0.0
    snaps = {}
    done = 0
    for n in segs:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        sim.step(n)
        torch.cuda.synchronize()
        seconds += time.perf_counter() - t0
        done += n
        snaps[done] = {c: sim.get_field(c).astype(np.float64) for c in ("ex", "ey", "ez", "bx", "by", "bz")}
    tm = sim.timers()
    d = sim.diagnostics()
    kin = d["kinetic_fraction"]
    sim.close()
    return {"seconds": seconds, "timers": tm, "diag": d, "snaps": snaps, "kinetic_fraction": kin}


def warm_up(cfg, steps, precision):
    """Untimed warm-up: the same configuration on a throwaway simulation."""
    import torch

    from paper_2510_11174_amd import hk
    sim = hk.Sim(cfg, precision=precision)
    sim.step(steps)
    torch.cuda.synchronize()
    sim.close()


def total_energy(d):
    return (d["u_e"] + d["u_b"] + sum(d["kin"]) + sum(d["fluid_kin"]) + d["conv_loss"]
            + d["ion_energy"] + d["photon_energy"])


def cpu_baseline(warm=60, timed=50):
    """FP64 oracle on a 64 x 32 x 32 crop of the same physics (threshold switch),
    single thread; steps/s scaled to the full grid by the cell ratio."""
    import oracle
    from paper_2510_11174_amd import configs
    oracle.build(force=False)
    cfg = configs.ionization_hybrid(64, 32, 32, mode="threshold")
    o = oracle.Oracle(cfg)
    o.step(warm)
    n = o.count(0)
    t0 = time.perf_counter()
    o.step(timed)
    dt = time.perf_counter() - t0
    full_cells = 128 * 64 * 64
    crop_cells = 64 * 32 * 32
    return {"value": timed / dt * crop_cells / full_cells, "unit": "steps/s", "cores": 1,
            "kind": "oracle",
            "sample": "FP64 oracle, 64x32x32 crop of the ionizing-helium case, threshold switch, "
                      "steps %d-%d, %.1f s; steps/s scaled by the cell ratio %d" % (
                          warm, warm + timed, dt, full_cells // crop_cells),
            "pushes_per_s": n * timed / dt}


MFMA_BF16_PEAK_TFLOPS = 2500.0   # MI355X dense BF16


def cnn_inference(reps=20):
    """One learned-switch evaluation's network pass on the ionizing-helium node
    grid (129 x 64 x 64 nodes with the 4-node halo), timed with HIP events on
    the library stream; flops are those of the four valid convolutions and the head."""
    import numpy as np
    import torch

    from paper_2510_11174_amd import hk
    from paper_2510_11174_amd import train as T
    D, H, W = 64 + 8, 64 + 8, 129 + 8
    cnn = hk.CNN(seed=1)
    cnn.set_params(T.init_params(1))
    x = torch.randn((1, D, H, W, 8), device="cuda", dtype=torch.float32)
    flops = 0
    for l, cin in enumerate((8, 32, 32, 32)):
        flops += 2 * 27 * cin * 32 * (D - 2 * l - 2) * (H - 2 * l - 2) * (W - 2 * l - 2)
    flops += 2 * 32 * (D - 8) * (H - 8) * (W - 8)
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
            "frac": round(tf / MFMA_BF16_PEAK_TFLOPS, 4), "kernel": "k_conv_fwd (4 layers) + k_head",
            "ms_per_eval": round(ms, 3), "flop_per_eval": flops,
            "grid": "129 x 64 x 64 nodes + halo 4"}


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
    bytes per node and step: read n, u, E, B, J and write n, u, J (20 values),
    plus read and write S for the warm fluid (22), in the build's real type."""
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
        alg = (22 if ga > 0 else 20) * 4 * nodes
        gbs = alg / (ms * 1e-3) / 1e9
        out[name] = {"ms_fluid_per_step": round(ms, 4), "alg_bytes_per_step": alg,
                     "achieved": round(gbs, 1), "frac": round(gbs / HBM_PEAK_GBS, 4),
                     "steps_per_s": round(steps / sec, 1), "fluid_heat": d["fluid_th"][0]}
    w = out["warm"]
    traffic = measured_traffic(FLUID_TRAFFIC_FILE, FLUID_SOURCES, "bytes_per_step_warm")
    return {"bound": "hbm", "achieved": w["achieved"], "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": w["frac"],
            "traffic": traffic, "kernel": "k_fluid_lorentz + k_fluid_update (warm)", "nodes": nodes,
            "workload": "plain plasma %dx%dx%d, all fluid, u_th 0.05" % (nx, ny, nz), **{k: v for k, v in out.items()}}


def field_l2(x, y):
    import numpy as np
    num = math.sqrt(sum(float(np.sum((x[c] - y[c]) ** 2)) for c in x))
    den = math.sqrt(sum(float(np.sum(y[c] ** 2)) for c in y))
    return num / den if den > 0 else 0.0


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=2000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--modes", default="threshold,all_pic",
                    help="comma list of switch modes to run (profiling runs may pick one)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="only run a 1 GiB device copy (counter calibration) and exit")
    ap.add_argument("--warm-fluid-only", action="store_true",
                    help="only measure the fluid phase (warm and cold) on the all-fluid 256x128x128 plasma")
    ap.add_argument("--networks-only", action="store_true",
                    help="only measure the next-state surrogate (64 patches of 16^3) and SwitchNet (the "
                         "ionizing-helium node grid) and print their JSON")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path (domain decomposition) is not "
              "implemented by this library; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2510_11174_amd import configs
    if args.networks_only:
        print(json.dumps({"roofline_state_predictor": sp_surrogate(), "roofline_switchnet": swn_inference()}))
        return
    if args.calibrate_copy:
        copy_calibration()
        return
    if args.warm_fluid_only:
        print(json.dumps({"roofline_warm_fluid": warm_fluid()}))
        return

    W, K = args.warmup, args.steps
    half = K // 2 if K >= 2 else None
    modes = [m for m in args.modes.split(",") if m]
    if any(m not in ("threshold", "all_pic") for m in modes) or not modes:
        print("--modes takes threshold and/or all_pic", file=sys.stderr)
        sys.exit(2)
    res = {}
    for mode in modes:
        cfg = configs.ionization_hybrid(mode=mode)
        print("bench: %s %s warm-up %d, timed steps 0-%d" % (cfg["name"], mode, W, K), file=sys.stderr,
              flush=True)
        if W > 0:
            warm_up(cfg, W, args.precision)
        res[mode] = run_gpu(cfg, K, args.precision, snap_at=half)
    if len(res) < 2:
        r = next(iter(res.values()))
        print(json.dumps({"mode": modes[0], "steps_per_s": K / r["seconds"], "timers": r["timers"]}))
        return
    h, p = res["threshold"], res["all_pic"]
    # the same all-PIC run again: FP32 atomics make the sums order dependent,
    # so two identical runs differ; this is the floor of any comparison
    print("bench: all-PIC repeat (run-to-run floor)", file=sys.stderr, flush=True)
    p2 = run_gpu(configs.ionization_hybrid(mode="all_pic"), K, args.precision, timing=False, snap_at=half)
    hyb_sps = K / h["seconds"]
    pic_sps = K / p["seconds"]
    l2 = {s: field_l2(h["snaps"][s], p["snaps"][s]) for s in p["snaps"]}
    floor = {s: field_l2(p2["snaps"][s], p["snaps"][s]) for s in p["snaps"]}
    e_h, e_p = total_energy(h["diag"]), total_energy(p["diag"])
    drift = abs(e_h - e_p) / abs(e_p) if e_p else 0.0
    traffic = measured_traffic()

    def roof(r, with_traffic):
        tm = r["timers"]
        ms = tm["push_kernel_ms"]
        alg = BYTES_PER_PUSH * tm["particles_pushed"] + BYTES_PER_TILE_CELL * TILE_CELLS * tm["tiles_pushed"]
        launches = max(tm["push_launches"], 1)
        achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": traffic if with_traffic else None,
                "kernel": "k_push", "avg_launch_ms": round(ms / launches, 4),
                "alg_bytes_per_launch": round(alg / launches)}

    out = {
        "metric": "hybrid steps/s vs all-PIC on same GPU at field err <=1e-3; particle pushes/s",
        "value": round(hyb_sps, 2),
        "unit": "steps/s",
        "n_gpus": 1,
        "steps": K,
        "warmup": W,
        "ms_per_step": round(1e3 / hyb_sps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32" if args.precision == "f32" else "f64",
        "data": "synthetic",
        "config": {"workload": "ionizing helium 128x64x64, dx 0.1, 8 ppc, a0 10, threshold switch "
                               "vs all-PIC, steps 0-%d from t = 0" % K,
                   "grid": [128, 64, 64], "ppc": 8, "switch": "threshold"},
        "allpic_steps_per_s": round(pic_sps, 2),
        "speedup_vs_allpic": round(hyb_sps / pic_sps, 3),
        "pushes_per_s": round(h["timers"]["particles_pushed"] / h["seconds"], 1),
        "allpic_pushes_per_s": round(p["timers"]["particles_pushed"] / p["seconds"], 1),
        "cell_steps_per_s": round(128 * 64 * 64 * hyb_sps, 1),
        "field_rel_l2_vs_allpic": {str(k): v for k, v in l2.items()},
        "field_rel_l2_allpic_repeat": {str(k): v for k, v in floor.items()},
        "energy_diff_vs_allpic": drift,
        # the hybrid meets 1e-3 at every snapshot where two all-PIC runs agree to
        # 1e-3; where they do not (FP32 atomics and a chaotic plasma), it must lie
        # within 10% of their distance, a single sample of the run-to-run noise
        "field_err_ok": all(l2[s] <= 1e-3 if floor[s] <= 1e-3 else l2[s] <= 1.1 * floor[s] for s in l2),
        "field_err_over_floor": {str(k): round(l2[k] / floor[k], 4) if floor[k] > 0 else None for k in l2},
        "kinetic_fraction_end": h["kinetic_fraction"],
        "roofline": roof(p, True),
        "roofline_hybrid": roof(h, False),
        "timers_hybrid_ms_per_step": {k: round(v / K, 4) for k, v in h["timers"].items() if k.endswith("_ms")},
        "timers_allpic_ms_per_step": {k: round(v / K, 4) for k, v in p["timers"].items() if k.endswith("_ms")},
        "rebins": {"hybrid": h["timers"]["rebins"], "all_pic": p["timers"]["rebins"]},
    }
    # the field update (Yee, Mur walls, antenna) of the all-PIC run, from its
    # HIP-event phase timer; algorithmic bytes per cell and step: read E, B and
    # write B, then read E, B, J and write E (84 B; the two B half steps that
    # give B at whole steps for the push move 120 B)
    cells = 128 * 64 * 64
    f_ms = p["timers"]["fields_ms"] / K
    yee_gbs = 84 * cells / (f_ms * 1e-3) / 1e9 if f_ms > 0 else 0.0
    out["roofline_yee"] = {"bound": "hbm", "achieved": round(yee_gbs, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": round(yee_gbs / HBM_PEAK_GBS, 4), "traffic": None,
                           "kernel": "k_b_half x2 + k_e_full + k_mur_save + k_mur_apply + k_antenna",
                           "ms_per_step": round(f_ms, 4), "alg_bytes_per_step": 84 * cells}
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
