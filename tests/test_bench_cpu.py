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


def _write_csv(path, header, rows):
    import csv
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(header)
        w.writerows(rows)


def test_trace_summary_takes_last_dispatches(tmp_path, capsys):
    # k_push dispatches of 10 us, then 20 us; the last two average 20 us, and
    # a kernel whose name only starts with k_push is not counted
    d = tmp_path / "trace" / "host"
    rows = [["KERNEL_DISPATCH", i, "void (anonymous namespace)::k_push<%d>(SpecP)" % (i % 2), 1000 * i,
             1000 * i + (10000 if i < 3 else 20000)] for i in range(5)]
    rows.append(["KERNEL_DISPATCH", 9, "(anonymous namespace)::k_push_other(int)", 0, 999999])
    _write_csv(d / "run_kernel_trace.csv", ["Kind", "Dispatch_Id", "Kernel_Name", "Start_Timestamp",
                                            "End_Timestamp"], rows)
    _write_csv(d / "run_kernel_stats.csv", ["Name", "Calls", "TotalDurationNs", "AverageNs"],
               [["k_push", 5, 70000, 14000], ["k_push_other", 1, 999999, 999999]])
    bench.summarize_trace(str(tmp_path / "trace"), "k_push", 2)
    out = capsys.readouterr().out
    assert "5 dispatches in the run; the last 2: mean 20.0 us" in out


def test_traffic_summary_scales_by_copy(tmp_path, capsys):
    # the copy reads half of 1 GiB on FETCH_SIZE: fetch is scaled by 2
    hdr = ["Dispatch_Id", "Kernel_Name", "Counter_Name", "Counter_Value"]
    gib_kib = 1024 * 1024
    _write_csv(tmp_path / "cf" / "run_counter_collection.csv", hdr,
               [[1, "fill_kernel", "FETCH_SIZE", 10], [2, "copyBuffer", "FETCH_SIZE", gib_kib / 2]])
    _write_csv(tmp_path / "cw" / "run_counter_collection.csv", hdr,
               [[1, "fill_kernel", "WRITE_SIZE", gib_kib], [2, "copyBuffer", "WRITE_SIZE", gib_kib]])
    _write_csv(tmp_path / "f" / "run_counter_collection.csv", hdr,
               [[i, "k_push(SpecP)", "FETCH_SIZE", 100 if i < 2 else 200] for i in range(4)])
    _write_csv(tmp_path / "w" / "run_counter_collection.csv", hdr,
               [[i, "k_push(SpecP)", "WRITE_SIZE", 50] for i in range(4)])

    class A:
        fetch, write = str(tmp_path / "f"), str(tmp_path / "w")
        calib_fetch, calib_write = str(tmp_path / "cf"), str(tmp_path / "cw")
        kernel, last, alg_bytes, window = "k_push", 2, 409600.0, "a0 5, steps 1-2"
    bench.summarize_traffic(A)
    kv = dict(l.split(" = ", 1) for l in capsys.readouterr().out.splitlines() if " = " in l and l[0] != "#")
    assert float(kv["fetch_bytes_per_launch"]) == 200 * 1024 * 2
    assert float(kv["write_bytes_per_launch"]) == 50 * 1024
    assert float(kv["traffic_over_algorithmic"]) == 1.125
    assert kv["window"] == "a0 5, steps 1-2" and kv["source_hash"] == bench.source_hash()
