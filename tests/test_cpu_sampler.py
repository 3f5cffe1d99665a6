"""CPU RadiusFPS product path (rfps_cpu_sample) against the oracle.

The entry point runs on the host only, so these tests run without a GPU.
Bar: bit-exact indices and FP32 distances for every grid, tile size and team
size (all output-neutral), in both distance forms; errors reported as
documented."""
import numpy as np
import pytest

import synth


@pytest.fixture(scope="module")
def rf():
    import paper_2606_06255_amd as rf
    return rf


def same(got, ref, what=""):
    gi, gd = got
    ri, rd = ref
    bad = np.flatnonzero(gi != ri)
    assert bad.size == 0, "%s: first index mismatch at %d: %d vs %d" % (what, bad[0], gi[bad[0]], ri[bad[0]])
    bd = np.flatnonzero(gd.view(np.uint32) != rd.view(np.uint32))
    assert bd.size == 0, "%s: first distance mismatch at %d: %r vs %r" % (what, bd[0], gd[bd[0]], rd[bd[0]])


def test_cube_partitions_and_teams(rf, oracle_lib):
    P = synth.cube(1)
    ref = oracle_lib.fps(P, 1024, 3)
    ref_eu = oracle_lib.fps(P, 1024, 3, euclid=True)
    for threads in (1, 2, 5, 16):
        for n_vox in (1, 3, 16, 100):
            for tile in (0, 1, 7):
                what = "threads=%d n_vox=%d tile=%d" % (threads, n_vox, tile)
                same(rf.cpu_fps(P, 1024, 3, n_vox=n_vox, tile=tile, threads=threads), ref, what)
        same(rf.cpu_fps(P, 1024, 3, threads=threads, flags=rf.F_SQRT), ref_eu, "euclid threads=%d" % threads)


def test_room_full(rf, oracle_lib):
    P = synth.room(0)
    ref = oracle_lib.fps(P, 20000, 0, threads=0)
    same(rf.cpu_fps(P, 20000, 0, threads=4), ref, "room default grid")
    same(rf.cpu_fps(P, 20000, 0, n_vox=24, threads=3), ref, "room n_vox=24")


def test_lidar_stage(rf, oracle_lib):
    P = synth.lidar(2)
    ref = oracle_lib.fps(P, 7164, 0, threads=0)
    same(rf.cpu_fps(P, 7164, 0, n_vox=32, threads=4), ref, "lidar")


def test_grid_rounding_ties_euclid(rf, oracle_lib):
    rng = np.random.default_rng(3)
    P = rng.integers(-30, 31, size=(8000, 3)).astype(np.float32) * np.float32(0.1)
    ref_eu = oracle_lib.fps(P, 2500, 0, threads=0, euclid=True)
    ref_sq = oracle_lib.fps(P, 2500, 0, threads=0)
    assert not np.array_equal(ref_eu[0], ref_sq[0])
    same(rf.cpu_fps(P, 2500, 0, flags=rf.F_SQRT, threads=4), ref_eu, "euclid")
    same(rf.cpu_fps(P, 2500, 0, threads=4), ref_sq, "squared")


def test_edge_cases(rf, oracle_lib):
    rng = np.random.default_rng(12)
    cases = [
        ("n1", np.zeros((1, 3), np.float32), 1, 0),
        ("m_eq_n", synth.cube(2)[:300], 300, 299),
        ("identical", np.ones((500, 3), np.float32), 50, 3),
        ("duplicates", np.repeat(synth.cube(3)[:200], 5, axis=0), 600, 0),
        ("lattice_ties", np.stack(np.meshgrid(*[np.arange(8)] * 3, indexing="ij"), -1)
         .reshape(-1, 3).astype(np.float32), 512, 0),
        ("planar", np.c_[rng.random((3000, 2)), np.zeros(3000)].astype(np.float32), 1500, 7),
        ("wide_range", (rng.normal(size=(2000, 3)) * 1e4).astype(np.float32), 1000, 0),
        ("tiny_scale", (rng.random((2000, 3)) * 1e-6).astype(np.float32), 1000, 0),
    ]
    for name, P, m, s in cases:
        ref = oracle_lib.fps(P, m, s)
        for threads in (1, 3):
            same(rf.cpu_fps(P, m, s, threads=threads), ref, "%s threads=%d" % (name, threads))
            same(rf.cpu_fps(P, m, s, n_vox=64, threads=threads), ref, "%s n_vox=64 threads=%d" % (name, threads))


def test_more_threads_than_tiles(rf, oracle_lib):
    P = synth.cube(4, 100)
    same(rf.cpu_fps(P, 100, 0, threads=64), oracle_lib.fps(P, 100, 0), "64 threads, 2 tiles")


def test_errors(rf):
    P = synth.cube(0)
    with pytest.raises(rf.RfpsError) as e:
        rf.cpu_fps(P, 5000, 0)
    assert e.value.status == 1
    with pytest.raises(rf.RfpsError):
        rf.cpu_fps(P, 10, 4096)
    with pytest.raises(rf.RfpsError):
        rf.cpu_fps(P, 10, 0, n_vox=2000)
    with pytest.raises(rf.RfpsError):
        rf.cpu_fps(P, 10, 0, flags=rf.F_UNFUSED)
    Q = P.copy()
    Q[7, 1] = np.inf
    with pytest.raises(rf.RfpsError) as e:
        rf.cpu_fps(Q, 10, 0)
    assert e.value.status == 2


@pytest.mark.parametrize("seed", range(6))
def test_random_configurations(rf, oracle_lib, seed):
    # seeded clouds of several shapes, sizes, starts, grids, tiles, team sizes
    # and both distance forms
    rng = np.random.default_rng(3000 + seed)
    for case in range(6):
        n = int(np.exp(rng.uniform(np.log(2), np.log(6000))))
        kind = int(rng.integers(0, 5))
        if kind == 0:
            P = rng.random((n, 3))
        elif kind == 1:
            P = rng.integers(-10, 11, size=(n, 3)) * 0.1
        elif kind == 2:
            base = rng.random((max(1, n // 3), 3))
            P = base[rng.integers(0, len(base), n)]
        elif kind == 3:
            P = np.c_[rng.random((n, 2)), np.zeros(n)]
        else:
            P = rng.normal(size=(n, 3)) * 10.0 ** rng.integers(-3, 5)
        P = np.ascontiguousarray(P.astype(np.float32))
        m = int(rng.integers(1, n + 1))
        start = int(rng.integers(0, n))
        euclid = bool(rng.integers(0, 3) == 0)
        n_vox = int(rng.choice([0, 1, 3, 24, 200]))
        tile = int(rng.choice([0, 1, 5, 64]))
        threads = int(rng.choice([1, 2, 3, 8]))
        ref = oracle_lib.fps(P, m, start, euclid=euclid)
        got = rf.cpu_fps(P, m, start, n_vox=n_vox, tile=tile, threads=threads, flags=rf.F_SQRT if euclid else 0)
        same(got, ref, "seed %d case %d kind %d n %d m %d n_vox %d tile %d threads %d euclid %s" % (
            seed, case, kind, n, m, n_vox, tile, threads, euclid))
