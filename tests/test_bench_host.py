"""Host logic of bench.py that needs no GPU: the one-GPU contract, option
checks, and the rule that stored counter traffic is only reported for the
sources it was measured on."""
import json
import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def run(*args):
    return subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), *args], capture_output=True,
                          text=True, timeout=300, cwd=ROOT)


def test_more_than_one_gpu_is_refused():
    r = run("--gpus", "2")
    assert r.returncode == 2
    assert "exactly one GPU" in r.stderr
    assert r.stdout == ""


def test_euclid_only_for_single_clouds():
    for w in ("batch", "lidar_stages"):
        r = run("--distance", "euclid", "--workload", w)
        assert r.returncode == 2 and "single-cloud" in r.stderr


def test_stored_traffic_follows_the_source_digest(tmp_path, monkeypatch):
    sys.path.insert(0, ROOT)
    import bench
    d = bench.source_digest()
    assert d == bench.source_digest() and len(d) == 16
    rec = json.load(open(os.path.join(ROOT, "profiles", "traffic.json")))["dense_lidar"]
    got = bench.stored_traffic("dense_lidar", rec["source_digest"])
    assert got == rec["bytes_per_launch"]
    assert bench.stored_traffic("dense_lidar", "0" * 16) is None
    assert bench.stored_traffic("no_such_workload", rec["source_digest"]) is None
