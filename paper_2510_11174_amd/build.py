"""Build the gfx950 C-ABI libraries in-tree: libhk_f32.so and libhk_f64.so.

Every source under csrc/ is compiled by hipcc for gfx950 twice (HK_DOUBLE off
and on) and linked into one shared library per precision.  Packed FP32 ops are
disabled (-packed-fp32-ops) and global float atomics are native
(-munsafe-fp-atomics; all device memory is coarse-grained).
"""
from __future__ import annotations

import concurrent.futures as cf
import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
BUILD = os.path.join(HERE, "_build")
SOURCES = ["k_fields.hip", "k_particles.hip", "k_diag.hip", "k_fluid.hip", "k_switch.hip", "hk_qed.cpp", "k_cnn.hip", "hk_cnn.cpp",
           "k_sp.hip", "hk_sp.cpp", "hk_swn.cpp", "k_dataset.hip", "hk_dataset.cpp", "hk_api.cpp"]
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
COMMON = ["-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950", "-munsafe-fp-atomics",
          "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-Wall", "-Wno-unused-function", "-Wno-unused-variable"]


def lib_path(prec: str) -> str:
    return os.path.join(HERE, "libhk_%s.so" % prec)


def _compile(src: str, prec: str) -> str:
    os.makedirs(os.path.join(BUILD, prec), exist_ok=True)
    obj = os.path.join(BUILD, prec, os.path.basename(src) + ".o")
    defs = ["-DHK_DOUBLE"] if prec == "f64" else []
    cmd = [HIPCC] + COMMON + defs + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        raise RuntimeError("hipcc failed for %s (%s):\n%s" % (src, prec, r.stderr[-6000:]))
    return obj


def build(precisions=("f32", "f64"), jobs: int | None = None) -> list[str]:
    jobs = jobs or min(8, os.cpu_count() or 4)
    srcs = [s for s in SOURCES if os.path.exists(os.path.join(CSRC, s))]
    with cf.ThreadPoolExecutor(jobs) as ex:
        futs = {(s, p): ex.submit(_compile, s, p) for p in precisions for s in srcs}
        objs = {k: f.result() for k, f in futs.items()}
    out = []
    for p in precisions:
        target = lib_path(p)
        tmp = target + ".tmp%d" % os.getpid()
        cmd = [HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC", "-o", tmp] + \
              [objs[(s, p)] for s in srcs]
        r = subprocess.run(cmd, capture_output=True, text=True)
        if r.returncode != 0:
            raise RuntimeError("link failed (%s):\n%s" % (p, r.stderr[-4000:]))
        os.replace(tmp, target)
        out.append(target)
    return out


if __name__ == "__main__":
    precs = tuple(sys.argv[1:]) or ("f32", "f64")
    for p in build(precs):
        print(p)
