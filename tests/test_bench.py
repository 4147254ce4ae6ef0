"""Host-side parts of bench.py (no GPU): the algorithmic byte counts of the
passes at the benchmark size, the lookup of the committed counter traffic,
and the single-GPU guard."""

import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import bench  # noqa: E402


def test_algorithmic_bytes_pillars():
    n = (320, 320, 48)
    # one complex FP32 value = 8 bytes; spectra after the x pass (3 x 48 x 320 x 321),
    # after the y pass (3 x 48 x 640 x 321); Lambda octant 6 x 49 x 321 x 321 FP32
    a = 3 * 48 * 320 * 321 * 8
    b = 3 * 48 * 640 * 321 * 8
    lam = 6 * 49 * 321 * 321 * 4
    assert bench.algorithmic_bytes("z_fused", n, 4, 4, 52) == 2 * b + lam == 594509976
    assert bench.algorithmic_bytes("y_forward", n, 4, 4, 52) == a + b
    f = 3 * 96 * 640 * 321 * 8
    assert bench.algorithmic_bytes("history_mac", n, 4, 4, 52, blk=8) == 52 * (f + lam) + 8 * f
    # far lags by FFTs in time, two earlier blocks of 32 steps: 64 spectra
    # read, 2 x 33 frequencies of the complex lag-segment spectra, 32 written
    assert bench.algorithmic_bytes("history_far", n, 4, 4, 2, blk=32) == 64 * f + 2 * 33 * 2 * lam + 32 * f


def test_measured_traffic_lookup():
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    recs = json.load(open(path))
    assert recs, "no counter records"
    for key, rec in recs.items():
        kernel, v = key.rsplit("/v", 1)
        assert rec["tile_variant"] == int(v)
        got = bench.measured_traffic(kernel, int(v))
        if bench.sources_sha256(rec["sources"]) == rec["sources_sha256"]:
            assert got == rec["bytes_per_launch"]
        else:
            assert got is None  # taken before a source change: not reported
    assert bench.measured_traffic("no_such_kernel", 0) is None


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode == 2
    assert "single-GPU" in r.stderr


def test_counter_summary(tmp_path):
    # per-kernel averages of a --pmc counter; dispatches under 20 % of the
    # kernel's median (behind a closed convergence gate) are left out
    d = tmp_path / "pmc" / "host"
    d.mkdir(parents=True)
    rows = [("k_a", 100.0), ("k_a", 110.0), ("k_a", 1.0), ("k_b", 50.0)]
    with open(d / "run_counter_collection.csv", "w") as f:
        f.write("Kernel_Name,Grid_Size,Counter_Name,Counter_Value\n")
        for k, v in rows:
            f.write(f"{k},256,FETCH_SIZE,{v}\n")
        f.write("k_a,256,WRITE_SIZE,999\n")
        f.write("k_a,512,FETCH_SIZE,7\n")
    out = bench.counter_summary(str(tmp_path / "pmc"), "FETCH_SIZE")
    assert out["k_a|256"]["kib"] == 105.0 and out["k_a|256"]["dispatches"] == 2
    assert out["k_a|256"]["all_dispatches"] == 3
    assert out["k_b|256"]["kib"] == 50.0 and out["k_a|512"]["kib"] == 7.0
