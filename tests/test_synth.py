"""Seeded generators: same seed gives the same bytes; shapes and ranges of each workload."""
import json
import os

import numpy as np

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden", "synth_sha256.json")


def test_fingerprints_pinned():
    ref = json.load(open(GOLD))
    for s in (0, 1):
        assert synth.fingerprint(synth.cube(s)) == ref["cube_%d" % s]
        assert synth.fingerprint(synth.room(s)) == ref["room_%d" % s]
        assert synth.fingerprint(synth.lidar(s)) == ref["lidar_%d" % s]
    xyz, off, m = synth.batch(0)
    assert synth.fingerprint(xyz) == ref["batch_0"]
    assert off.tolist() == ref["batch_0_offsets"]


def test_cube_shape():
    a = synth.cube(3)
    assert a.shape == (4096, 3) and a.dtype == np.float32
    assert a.min() >= 0.0 and a.max() < 1.0
    assert not np.array_equal(a, synth.cube(4))


def test_room_shape_and_extent():
    r = synth.room(0)
    assert r.shape == (synth.ROOM_N, 3) and r.dtype == np.float32
    lo, hi = r.min(0), r.max(0)
    assert np.all(lo > -0.05) and np.all(hi < np.array([10.05, 8.05, 3.05]))
    # floor and ceiling both populated
    assert (np.abs(r[:, 2]) < 0.02).sum() > 1000
    assert (np.abs(r[:, 2] - 3.0) < 0.02).sum() > 1000


def test_lidar_shape_and_scene():
    l = synth.lidar(0)
    assert l.shape == (synth.LIDAR_N, 3) and l.dtype == np.float32
    rng_h = np.hypot(l[:, 0], l[:, 1])
    assert rng_h.max() < 80.3                     # far wall
    assert (np.abs(l[:, 2] + 1.7) < 0.1).sum() > 20000  # ground returns
    assert synth.lidar_stage_sizes() == [114624, 28656, 7164, 1791]


def test_dense_lidar_size():
    # generator arithmetic only (no sampling): 128 x 8192 returns
    d = synth.lidar(0, beams=128, azimuth_steps=8192, drop=0)
    assert d.shape == (synth.DENSE_N, 3)


def test_batch_sizes():
    xyz, off, m = synth.batch(0)
    n = np.diff(off)
    assert len(n) == 32 and n.min() >= 8000 and n.max() <= 120000
    assert np.array_equal(m, n // 4)
    assert xyz.shape[0] == off[-1]
