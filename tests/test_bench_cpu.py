"""bench.py's host-side contract, on the CPU: it refuses more than one GPU
before touching a device, it reports the committed HBM traffic of a kernel
only while the kernel sources and the launch's cell count are those the
counters were taken for, and every committed traffic summary carries the
fields it reads."""
import glob
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""


def test_traffic_is_reported_only_for_the_current_kernels(tmp_path):
    path = tmp_path / "traffic_k_w_f32.txt"

    def write(h, cells):
        path.write_text(f"# a summary\nkernel_hash = {h}\ncells_per_launch = {cells}\n"
                        f"bytes_per_launch = 4567\nalgorithmic_bytes_per_launch = 4000\n")

    write(bench.kernel_hash(), 123)
    assert bench.measured_traffic(str(path), 123) == 4567
    assert bench.measured_traffic(str(path), 124) is None      # another launch shape
    write("0" * 16, 123)
    assert bench.measured_traffic(str(path), 123) is None      # kernels changed since
    assert bench.measured_traffic(str(tmp_path / "missing.txt"), 123) is None


def test_committed_traffic_summaries_parse():
    files = sorted(glob.glob(os.path.join(ROOT, "profiles", "traffic_*.txt")))
    assert files
    for f in files:
        vals = {}
        for line in open(f):
            line = line.split("#", 1)[0].strip()
            if "=" in line:
                k, v = line.split("=", 1)
                vals[k.strip()] = v.strip()
        for k in ("kernel_hash", "cells_per_launch", "bytes_per_launch", "algorithmic_bytes_per_launch"):
            assert k in vals, (f, k)
        ratio = float(vals["bytes_per_launch"]) / float(vals["algorithmic_bytes_per_launch"])
        assert 1.0 <= ratio < 2.0, (f, ratio)   # every population is moved at least once
        assert len(vals["kernel_hash"]) == 16
