"""Host-side pieces of bench.py: the algorithmic bytes models, the rocprofv3 counter
digest and the traffic summary (synthetic counter files, no GPU)."""
import json
import os

import pytest

import bench


def _write_counters(d, rows):
    os.makedirs(d, exist_ok=True)
    with open(os.path.join(d, "run_counter_collection.csv"), "w") as f:
        f.write('"Correlation_Id","Dispatch_Id","Kernel_Name","Counter_Name","Counter_Value"\n')
        for i, (k, c, v) in enumerate(rows):
            f.write(f'{i},{i},"{k}","{c}",{v}\n')


def test_bytes_models():
    # rounds 2.. only; push: 20 B per worklist vertex
    assert bench.assign_bytes([10, 4, 2], [100, 40, 20], push=True) == 20 * 6
    assert bench.assign_bytes([10, 4, 2], [100, 40, 20], push=False) == 16 * 6 + 8 * 60
    # detect: 20 B/vertex + 8 B/examined arc + 4 B per requeued vertex (+ 20 B per pushed arc)
    assert bench.detect_bytes([10, 4, 2], [0, 7, 3], 50, push=False) == 20 * 4 + 56 + 8 + 20 * 2 + 24 + 0
    assert bench.detect_bytes([10, 4, 2], [0, 7, 3], 50, push=True, byte_flags=False) == 20 * 4 + 56 + 8 + 20 * 2 + 24 + 1000
    assert bench.detect_bytes([10, 4, 2], [0, 7, 3], 50, push=True) == 20 * 4 + 56 + 8 + 20 * 2 + 24 + 650


def test_digest_and_traffic_summary(tmp_path, monkeypatch, capsys):
    f, w, cf, cw = (str(tmp_path / x) for x in ("f", "w", "cf", "cw"))
    _write_counters(f, [("void csrcolor::k_detect(csrcolor::RoundArgs)", "FETCH_SIZE", 100.0),
                        ("void csrcolor::k_detect(csrcolor::RoundArgs)", "FETCH_SIZE", 300.0),
                        ("csrcolor::k_assign(csrcolor::RoundArgs)", "FETCH_SIZE", 10.0)])
    _write_counters(w, [("void csrcolor::k_detect(csrcolor::RoundArgs)", "WRITE_SIZE", 50.0),
                        ("void csrcolor::k_detect(csrcolor::RoundArgs)", "WRITE_SIZE", 50.0),
                        ("csrcolor::k_assign(csrcolor::RoundArgs)", "WRITE_SIZE", 4.0)])
    # copy probe of 1 MiB reading 2048 KiB and writing 1024 KiB per dispatch -> factors 2 and 1
    _write_counters(cf, [("void at::native::copy_kernel(int)", "FETCH_SIZE", 2048.0),
                         ("void at::native::copy_kernel(int)", "FETCH_SIZE", 3.0)])     # a small extra dispatch
    _write_counters(cw, [("void at::native::copy_kernel(int)", "WRITE_SIZE", 1024.0)])
    assert bench.digest_pmc(f) == 0
    dig = json.loads(capsys.readouterr().out)
    assert dig["kernels"]["k_detect"]["FETCH_SIZE"]["dispatches"] == 2
    assert dig["kernels"]["k_detect"]["FETCH_SIZE"]["per_dispatch"] == 200.0
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.traffic_summary("toy", f, w, cf, cw, copy_mib=1) == 0
    capsys.readouterr()
    t = json.load(open(tmp_path / "profiles" / "traffic_toy.json"))
    k = t["kernels"]["k_detect"]
    assert t["fetch_factor"] == 2.0 and t["write_factor"] == 1.0
    assert k["fetch_bytes_per_launch"] == 200.0 * 1024 / 2.0
    assert k["write_bytes_per_launch"] == 50.0 * 1024
    # the figure is reported only while the kernel sources are unchanged
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: t["source_sha256"])
    assert bench.measured_traffic("toy", "k_detect") == k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]
    monkeypatch.setattr(bench, "kernel_source_digest", lambda: "other")
    assert bench.measured_traffic("toy", "k_detect") is None


def test_multi_gpu_request_is_refused():
    import subprocess
    import sys
    r = subprocess.run([sys.executable, os.path.join(os.path.dirname(bench.__file__), "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0 and "one GPU" in r.stderr
