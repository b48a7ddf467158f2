#!/usr/bin/env python
"""Benchmark of the hybrid fluid-kinetic step on one MI355X.

Workload: the ionizing-helium case (128 x 64 x 64 cells, dx = 0.1, 8 particles
per cell, neutral He 0.1 n_c with a 10-lambda up-ramp, a0 = 10 linear pulse,
waist 6 lambda, duration 15, ADK/multiphoton ionization, threshold switch).
The same seed runs twice on the same GPU: hybrid (threshold switch) and
all-PIC (every node kinetic).  After W untimed warm-up steps, K steps are timed
with a device synchronisation on both sides.

The JSON line reports hybrid steps/s (value), all-PIC steps/s, the speed-up,
particle pushes/s, the field relative L2 and energy difference between the two
runs at the end, the push kernel's achieved HBM rate against the roofline
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


def run_gpu(cfg, steps, warmup, precision):
    import numpy as np
    import torch

    from paper_2510_11174_amd import hk
    sim = hk.Sim(cfg, precision=precision)
    sim.step(warmup)
    torch.cuda.synchronize()
    sim.enable_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    sim.step(steps)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    tm = sim.timers()
    d = sim.diagnostics()
    fields = {c: sim.get_field(c).astype(np.float64) for c in ("ex", "ey", "ez", "bx", "by", "bz")}
    sim.close()
    return {"seconds": t1 - t0, "timers": tm, "diag": d, "fields": fields}


def total_energy(d):
    return (d["u_e"] + d["u_b"] + sum(d["kin"]) + sum(d["fluid_kin"]) + d["conv_loss"]
            + d["ion_energy"] + d["photon_energy"])


def cpu_baseline(warm=60, timed=60):
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


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=800)
    ap.add_argument("--warmup", type=int, default=200)
    ap.add_argument("--precision", default="f32", choices=["f32", "f64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the multi-GPU path (domain decomposition) is not "
              "part of this build; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    from paper_2510_11174_amd import configs

    W, K = args.warmup, args.steps
    res = {}
    for mode in ("threshold", "all_pic"):
        cfg = configs.ionization_hybrid(mode=mode)
        print("bench: %s %s warmup %d steps %d" % (cfg["name"], mode, W, K), file=sys.stderr,
              flush=True)
        res[mode] = run_gpu(cfg, K, W, args.precision)
    h, p = res["threshold"], res["all_pic"]
    hyb_sps = K / h["seconds"]
    pic_sps = K / p["seconds"]
    num = math.sqrt(sum(float(np.sum((h["fields"][c] - p["fields"][c]) ** 2)) for c in h["fields"]))
    den = math.sqrt(sum(float(np.sum(p["fields"][c] ** 2)) for c in p["fields"]))
    field_l2 = num / den if den > 0 else 0.0
    e_h, e_p = total_energy(h["diag"]), total_energy(p["diag"])
    drift = abs(e_h - e_p) / abs(e_p) if e_p else 0.0

    def roof(r):
        tm = r["timers"]
        ms = tm["push_kernel_ms"]
        alg = BYTES_PER_PUSH * tm["particles_pushed"] + BYTES_PER_TILE_CELL * TILE_CELLS * tm["tiles_pushed"]
        launches = max(tm["push_launches"], 1)
        achieved = alg / (ms * 1e-3) / 1e9 if ms > 0 else 0.0
        return {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
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
                               "vs all-PIC, steps %d-%d" % (W, W + K),
                   "grid": [128, 64, 64], "ppc": 8, "switch": "threshold"},
        "allpic_steps_per_s": round(pic_sps, 2),
        "speedup_vs_allpic": round(hyb_sps / pic_sps, 3),
        "pushes_per_s": round(h["timers"]["particles_pushed"] / h["seconds"], 1),
        "allpic_pushes_per_s": round(p["timers"]["particles_pushed"] / p["seconds"], 1),
        "field_rel_l2_vs_allpic": field_l2,
        "energy_diff_vs_allpic": drift,
        "field_err_ok": field_l2 <= 1e-3,
        "kinetic_fraction": h["diag"]["kinetic_fraction"],
        "roofline": roof(p),
        "roofline_hybrid": roof(h),
        "timers_hybrid_ms_per_step": {k: round(v / K, 4) for k, v in h["timers"].items() if k.endswith("_ms")},
        "timers_allpic_ms_per_step": {k: round(v / K, 4) for k, v in p["timers"].items() if k.endswith("_ms")},
        "rebins": {"hybrid": h["timers"]["rebins"], "all_pic": p["timers"]["rebins"]},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
