"""The benchmark's measurement logic on the CPU: the one-GPU rule, the
algorithmic work per launch behind the roofline, and the traffic record."""
import json
import os
import subprocess
import sys

import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in json.loads(r.stdout.strip().splitlines()[-1])["error"]


def test_tile_kernel_work_per_launch():
    """One read and one write of T per spin; flush of rank n_A plus the two
    panel products of depth k, per spin (40x40, N_sigma = 800, k = 32)."""
    p = synth.workload("c3")
    Ns, k, acc = 800, 32, 0.75
    flops, nbytes, bound = bench.kernel_work(p, "tile", "delayed", k, 16, acc)
    assert bound == "mfma"
    assert nbytes == 2 * 2 * Ns * Ns * 8
    assert flops == pytest.approx(2 * (2 * Ns * Ns * acc * k + 4 * Ns * Ns * k))


def test_roofline_fraction_from_launch_times():
    p = synth.workload("c3")
    ktimes = {"tile": (0.5, 5000), "decide": (0.1, 5000), "propagate": (0.2, 100)}
    r = bench.roofline(p, "delayed", 32, 16, 0.75, ktimes, walkers=8)
    flops, _, _ = bench.kernel_work(p, "tile", "delayed", 32, 16, 0.75)
    assert r["kernel"] == "tile" and r["unit"] == "TFLOP/s"
    assert r["achieved"] == pytest.approx(8 * flops / 1e-4 / 1e12)
    assert r["frac"] == pytest.approx(r["achieved"] / 78.6)
    assert sum(r["device_time_share"].values()) == pytest.approx(1.0)


def _record(cls):
    rec = {}
    path = bench.TRAFFIC_FILES[cls]
    if not os.path.exists(path):
        return None
    for line in open(path):
        if ":" in line and not line.startswith("#"):
            key, val = line.split(":", 1)
            rec[key.strip()] = val.strip()
    return rec


def test_traffic_record_matches_only_its_launch():
    """The committed rocprofv3 traffic covers the 8-walker k = 32 launch of the
    tile kernel and the 8-walker launch of the per-site local kernel on the
    40x40 workload while the kernel source is the one it was taken on (then it
    is the recorded figure, above the algorithmic bytes), and nothing else."""
    import hashlib
    src = os.path.join(ROOT, "paper_2506_09611_amd", "csrc", "update.hip")
    digest = hashlib.sha256(open(src, "rb").read()).hexdigest()
    for cls, scheme in (("tile", "delayed"), ("local", "local")):
        rec = _record(cls)
        t = bench.measured_traffic(cls, scheme, 32, 8, "c3")
        if rec is not None and rec["source_sha256"] == digest:
            assert t == float(rec["traffic_bytes_per_launch"])
            assert t > float(rec["algorithmic_bytes_per_launch"])
        else:
            assert t is None
        assert bench.measured_traffic(cls, scheme, 32, 4, "c3") is None
        assert bench.measured_traffic(cls, scheme, 32, 8, "c2") is None
    assert bench.measured_traffic("tile", "delayed", 16, 8, "c3") is None
    assert bench.measured_traffic("tile", "block", 32, 8, "c3") is None
    assert bench.measured_traffic("local", "delayed", 32, 8, "c3") is None
    assert bench.measured_traffic("decide", "delayed", 32, 8, "c3") is None
    rec = _record("tile")
    if rec is not None and "tile_chunks" in rec:
        c = int(rec["tile_chunks"])
        assert bench.measured_traffic("tile", "delayed", 32, 8, "c3", c + 1) is None
