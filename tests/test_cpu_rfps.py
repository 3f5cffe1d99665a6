"""CPU RadiusFPS (Sec. 3) against the plain oracle.

Pruning is conservative, so every voxel resolution, every split of voxels
into tiles, with or without the point skip, with the member radius or the
paper's sqrt(3)/2 L radius, must give the oracle's sequence bit for bit.
Planted mistakes (centroid-only pruning, a halved radius) must be caught.
"""
import numpy as np
import pytest

import synth


def bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(bits(a[1]), bits(b[1]))


def clouds():
    rng = np.random.default_rng(7)
    lat = np.stack(np.meshgrid(*[np.arange(9)] * 3, indexing="ij"), -1).reshape(-1, 3)
    sph = rng.normal(size=(3000, 3))
    sph /= np.linalg.norm(sph, axis=1, keepdims=True)
    corners = (rng.integers(0, 5, size=(3000, 3)) + rng.normal(0, 1e-4, size=(3000, 3)))
    return {
        "cube": (synth.cube(2), 1024),
        "room": (synth.room(4)[:15000], 2000),
        "lidar": (synth.lidar(4)[::6], 3000),
        "lattice": (lat.astype(np.float32), 729),
        "sphere_shells": (np.concatenate([sph * r for r in (1.0, 2.0, 3.0)]).astype(np.float32), 1500),
        "near_corners": (corners.astype(np.float32), 1500),
    }


@pytest.mark.parametrize("name", ["cube", "room", "lidar", "lattice", "sphere_shells", "near_corners"])
def test_partition_invariance(oracle_lib, name):
    P, m = clouds()[name]
    ref = oracle_lib.fps(P, m, 0)
    for n_vox in (1, 2, 3, 5, 8, 16, 24, 32, 64, 128):
        for tile in (0, 1, 5, 64):
            got = oracle_lib.rfps_cpu(P, m, 0, n_vox=n_vox, tile=tile)
            assert same(ref, got[:2]), (name, n_vox, tile)
    for opts in (oracle_lib.NO_SKIP, oracle_lib.PAPER_RADIUS, oracle_lib.NO_PRUNE,
                 oracle_lib.NO_SKIP | oracle_lib.PAPER_RADIUS):
        got = oracle_lib.rfps_cpu(P, m, 0, n_vox=16, tile=64, opts=opts)
        assert same(ref, got[:2]), (name, opts)


def test_start_indices(oracle_lib):
    P = synth.room(5)[:8000]
    for s in (0, 1, 4000, 7999):
        assert same(oracle_lib.fps(P, 700, s), oracle_lib.rfps_cpu(P, 700, s, n_vox=24)[:2])


def test_pruning_is_active(oracle_lib):
    P = synth.room(6)[:20000]
    _, _, tel = oracle_lib.rfps_cpu(P, 5000, 0, n_vox=24)
    assert tel["voxel_tests"] == tel["iters"] * tel["voxels"]
    assert tel["voxels_pruned"] > 0.9 * tel["voxel_tests"]
    assert tel["points_visited"] < 0.2 * tel["iters"] * P.shape[0]
    _, _, tel0 = oracle_lib.rfps_cpu(P, 5000, 0, n_vox=24, opts=oracle_lib.NO_PRUNE)
    assert tel0["points_visited"] == tel0["iters"] * P.shape[0]
    assert tel0["points_updated"] == tel["points_updated"]   # same strict decreases


@pytest.mark.parametrize("mut", ["MUT_CENTROID", "MUT_HALF_RADIUS"])
def test_planted_mistakes_are_caught(oracle_lib, mut):
    caught = 0
    for name, (P, m) in clouds().items():
        ref = oracle_lib.fps(P, m, 0)
        got = oracle_lib.rfps_cpu(P, m, 0, n_vox=8, opts=getattr(oracle_lib, mut))
        caught += not same(ref, got[:2])
    assert caught >= 3


def test_voxel_grid(oracle_lib):
    P = synth.room(0)
    for n_vox in (1, 7, 24, 128):
        pmin, L, vid = oracle_lib.voxelize(P, n_vox)
        assert np.array_equal(pmin, P.min(0).astype(np.float64))
        E = float((P.max(0).astype(np.float64) - pmin).max())
        assert L == pytest.approx((1 + 1e-4) * E / n_vox, rel=1e-15)
        v = np.stack([vid % n_vox, (vid // n_vox) % n_vox, vid // (n_vox * n_vox)], 1)
        assert v.max() < n_vox
        # every point lies in its cube (up to FP64 rounding of the quotient)
        lo = pmin + v * L
        assert np.all(P >= lo - 1e-9) and np.all(P <= lo + L + 1e-9)
    _, L, vid = oracle_lib.voxelize(np.ones((5, 3), np.float32), 16)
    assert L == 1.0 and np.all(vid == 0)
