"""Host logic of bench.py (no GPU): a profile summary taken on other kernel
sources (or missing) gives no measured traffic, and a request for several
GPUs exits with a message."""
import os

import bench


def test_stale_summary_is_refused(tmp_path):
    text = open(bench.FLUID_TRAFFIC_FILE).read()
    stale = tmp_path / "stale.txt"
    stale.write_text(text.replace("source_hash = ", "source_hash = 0"))
    assert bench.measured_traffic(str(stale), bench.FLUID_SOURCES, "bytes_per_step_warm") is None
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), bench.FLUID_SOURCES) is None


def test_multi_gpu_request_exits():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(bench.ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2 and "one GPU" in r.stderr
