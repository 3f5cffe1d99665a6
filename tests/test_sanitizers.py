"""Sanitizer builds of the host code, run on the CPU.

- The oracle (oracle/*.c) under AddressSanitizer + UndefinedBehaviorSanitizer,
  driven by tests/native/oracle_san_main.c: plain FPS, its Euclidean form and
  the oracle's CPU RadiusFPS over many grids and tile splits must agree.
- The library's host code (every source of librfps, the host side built with
  AddressSanitizer + UndefinedBehaviorSanitizer; the device code is compiled
  as usual and never launched) under tests/native/host_san_main.cpp: every
  entry point's host argument checks, and the CPU sampler against the oracle.
- The CPU sampler alone under ThreadSanitizer (its team meets in a lock-free
  exchange once per selection).

Each sanitizer aborts its process on the first error, so a non-zero exit code
is the failure.  The builds go to a temporary directory; nothing here touches
a GPU.
"""
import os
import shutil
import subprocess

import numpy as np
import pytest

import synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NATIVE = os.path.join(ROOT, "tests", "native")
CSRC = os.path.join(ROOT, "paper_2606_06255_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
LIB_SOURCES = ["rfps_api.hip", "index_build.hip", "sample_rfps.hip", "sample_rounds.hip", "sample_plain.hip",
               "sample_unfused.hip", "mlp.hip", "cpu_sampler.cpp"]
SAN_ENV = {
    "ASAN_OPTIONS": "detect_leaks=0:abort_on_error=0:halt_on_error=1",
    "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1",
    "TSAN_OPTIONS": "halt_on_error=1:second_deadlock_stack=1",
}


def _clouds():
    """(name, points, m): small clouds with ragged sizes, ties and duplicates."""
    rng = np.random.default_rng(7)
    lattice = np.stack(np.meshgrid(np.arange(5), np.arange(4), np.arange(3), indexing="ij"), -1)
    lattice = lattice.reshape(-1, 3).astype(np.float32)
    dup = np.repeat(rng.random((40, 3), dtype=np.float32), 3, axis=0)
    return [
        ("cube", synth.cube(1, n=700), 300),
        ("room", synth.room(2, n=2000), 500),
        ("lattice", lattice, len(lattice)),
        ("duplicates", dup, len(dup)),
        ("one", np.zeros((1, 3), np.float32), 1),
    ]


def _run(cmd, env=None, timeout=600):
    e = dict(os.environ)
    e.update(SAN_ENV)
    if env:
        e.update(env)
    r = subprocess.run(cmd, capture_output=True, text=True, env=e, timeout=timeout)
    assert r.returncode == 0, "%s\nexit %d\n%s\n%s" % (" ".join(cmd), r.returncode, r.stdout[-3000:],
                                                       r.stderr[-6000:])
    return r.stdout


def _write_cloud(tmp, name, P, m, oracle):
    cloud = os.path.join(tmp, name + ".f32")
    np.ascontiguousarray(P, np.float32).tofile(cloud)
    idx, d2 = oracle.fps(P, m, 0)
    ip, dp = os.path.join(tmp, name + ".idx"), os.path.join(tmp, name + ".d2")
    np.asarray(idx, np.int32).tofile(ip)
    np.asarray(d2, np.float32).tofile(dp)
    return cloud, ip, dp


@pytest.fixture(scope="module")
def clouds(tmp_path_factory, oracle_lib):
    tmp = str(tmp_path_factory.mktemp("san_clouds"))
    return [(name, m) + _write_cloud(tmp, name, P, m, oracle_lib) for name, P, m in _clouds()]


def test_oracle_asan_ubsan(tmp_path, clouds):
    exe = str(tmp_path / "oracle_san")
    srcs = [os.path.join(ROOT, "oracle", s) for s in ("fps_oracle.c", "cpu_rfps.c")]
    subprocess.run(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
                    "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer",
                    "-o", exe, os.path.join(NATIVE, "oracle_san_main.c"), *srcs, "-lm"], check=True)
    for name, m, cloud, _, _ in clouds:
        out = _run([exe, cloud, str(m), "0"], env={"OMP_NUM_THREADS": "2"})
        assert out.startswith("ok"), (name, out)


@pytest.mark.skipif(not os.path.exists(HIPCC), reason="hipcc not installed")
def test_library_host_asan_ubsan(tmp_path, clouds):
    # The host pass gets the sanitizers; the device pass is compiled at -O0
    # (its code is never launched here), which keeps the build short.
    exe = str(tmp_path / "host_san")
    cmd = [HIPCC, "--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-w",
           "-Xarch_device", "-O0",
           "-Xarch_host", "-fsanitize=address,undefined",
           "-Xarch_host", "-fno-sanitize-recover=all",
           "-Xarch_host", "-fno-omit-frame-pointer",
           "-o", exe, os.path.join(NATIVE, "host_san_main.cpp")] + [os.path.join(CSRC, s) for s in LIB_SOURCES]
    subprocess.run(cmd, check=True, timeout=900)
    for name, m, cloud, ip, dp in clouds:
        out = _run([exe, cloud, str(m), ip, dp])
        assert out.startswith("ok"), (name, out)


@pytest.mark.skipif(shutil.which("g++") is None, reason="g++ not installed")
def test_cpu_sampler_tsan(tmp_path, clouds):
    exe = str(tmp_path / "cpu_tsan")
    subprocess.run(["g++", "-O1", "-g", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-pthread",
                    "-fsanitize=thread", "-DCPU_SAMPLER_ONLY", "-Wno-unknown-pragmas", "-o", exe,
                    os.path.join(NATIVE, "host_san_main.cpp"), os.path.join(CSRC, "cpu_sampler.cpp")],
                   check=True)
    for name, m, cloud, ip, dp in clouds:
        out = _run([exe, cloud, str(m), ip, dp])
        assert out.startswith("ok"), (name, out)
