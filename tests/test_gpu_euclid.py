"""Euclidean distance mode (RFPS_F_SQRT) against the oracle's Euclidean FPS.

FPS over the FP32 norm differs from FPS over its square exactly where
rounding the root merges two squared distances into one value; the grid
clouds below (step 0.1, so many equal real distances with unequal FP32
squares) make that happen often, and the tests check that the two oracle
sequences really differ there before comparing the GPU with each."""
import numpy as np
import pytest
import torch

import oracle
import synth

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    import paper_2606_06255_amd as rf
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU")
    return rf


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def _same(got, ref, what):
    gi, gd = got[0].cpu().numpy(), got[1].cpu().numpy()
    ri, rd = ref
    bad = np.flatnonzero(gi != ri)
    assert bad.size == 0, "%s: first index mismatch at %d: %d vs %d" % (what, bad[0], gi[bad[0]], ri[bad[0]])
    bd = np.flatnonzero(gd.view(np.uint32) != rd.view(np.uint32))
    assert bd.size == 0, "%s: first distance mismatch at %d: %r vs %r" % (what, bd[0], gd[bd[0]], rd[bd[0]])


def grid_cloud(seed, n, half=40):
    rng = np.random.default_rng(seed)
    return rng.integers(-half, half + 1, size=(n, 3)).astype(np.float32) * np.float32(0.1)


def test_cube_partitions(rf):
    P = synth.cube(0)
    ref = oracle.fps(P, 1024, 0, euclid=True)
    x = dev(P)
    for n_vox in (4, 16):
        for tile in (0, 7):
            idx = rf.build_index(x, n_vox=n_vox, tile=tile)
            for g in (3, 64, 0):
                for la, fl in ((0, 0), (3, 0), (4, 0), (8, 0), (0, rf.F_SINGLE_PICK), (0, rf.F_NO_PRUNE),
                               (0, rf.F_NO_POINT_SKIP)):
                    got = rf.sample(idx, 1024, 0, groups=g, lookahead=la, flags=fl | rf.F_SQRT)
                    what = "n_vox=%d tile=%d g=%d lookahead=%d flags=%d" % (n_vox, tile, g, la, fl)
                    assert rf.read_status(idx) == 0, what
                    _same(got, ref, what)


@pytest.mark.parametrize("seed", [0, 1])
def test_grid_rounding_ties(rf, seed):
    P = grid_cloud(seed, 20000)
    M = 5000
    ref_eu = oracle.fps(P, M, 0, threads=0, euclid=True)
    ref_sq = oracle.fps(P, M, 0, threads=0)
    assert not np.array_equal(ref_eu[0], ref_sq[0])   # the case separates the two forms
    x = dev(P)
    idx = rf.build_index(x)
    for la in (2, 3, 4, 8):
        _same(rf.sample(idx, M, 0, lookahead=la, flags=rf.F_SQRT), ref_eu, "euclid lookahead %d" % la)
    _same(rf.sample(idx, M, 0, flags=rf.F_SQRT | rf.F_SINGLE_PICK), ref_eu, "euclid single pick")
    _same(rf.sample(idx, M, 0), ref_sq, "squared")


def test_wide_dynamic_range(rf):
    # one cluster whose squared distances are subnormal, one at 1e14 scale:
    # roots of values across the whole exponent range
    rng = np.random.default_rng(5)
    a = (rng.random((1500, 3)) * 1e-22).astype(np.float32)
    b = (rng.random((1500, 3)) * 1e14 + 1e14).astype(np.float32)
    c = rng.random((1000, 3)).astype(np.float32)
    P = np.concatenate([a, b, c])
    ref = oracle.fps(P, P.shape[0], 0, threads=0, euclid=True)
    x = dev(P)
    for la, fl in ((0, 0), (4, 0), (0, rf.F_SINGLE_PICK)):
        _same(rf.fps(x, P.shape[0], 0, lookahead=la, flags=fl | rf.F_SQRT), ref, "lookahead %d flags %d" % (la, fl))


def test_room_full(rf):
    P = synth.room(0)
    ref = oracle.fps(P, 20000, 0, threads=0, euclid=True)
    x = dev(P)
    _same(rf.fps(x, 20000, 0, flags=rf.F_SQRT), ref, "default")
    _same(rf.fps(x, 20000, 0, groups=256, lookahead=4, flags=rf.F_SQRT), ref, "g256 lookahead 4")


def test_lidar_stage(rf):
    P = synth.lidar(0)
    ref = oracle.fps(P, 28656, 0, threads=0, euclid=True)
    _same(rf.fps(dev(P), 28656, 0, flags=rf.F_SQRT), ref, "lidar stage 1")


@pytest.mark.parametrize("lookahead", [2, 8])
def test_batched(rf, lookahead):
    clouds = [grid_cloud(3, 3000), synth.cube(1, 700), synth.room(2, n=5000), synth.cube(4, 1),
              grid_cloud(4, 900, half=6)]
    sizes = [c.shape[0] for c in clouds]
    offsets = np.zeros(len(clouds) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    xyz = np.ascontiguousarray(np.concatenate(clouds).astype(np.float32))
    m = np.array([1500, 700, 1250, 1, 900], dtype=np.int32)
    ei, ed = [], []
    for c in range(len(m)):
        i, d = oracle.fps(xyz[offsets[c]:offsets[c + 1]], int(m[c]), 0, euclid=True)
        ei.append(i)
        ed.append(d)
    got = rf.sample_batched(dev(xyz), offsets, m, lookahead=lookahead, flags=rf.F_SQRT)
    _same(got, (np.concatenate(ei), np.concatenate(ed)), "batched lookahead %d" % lookahead)


def test_degenerate(rf):
    # identical points (all distances 0), two points, a single point
    for P, M in ((np.ones((100, 3), np.float32), 100), (np.array([[0, 0, 0], [3, 4, 0]], np.float32), 2),
                 (np.array([[1, 2, 3]], np.float32), 1)):
        ref = oracle.fps(P, M, 0, euclid=True)
        _same(rf.fps(dev(P), M, 0, flags=rf.F_SQRT), ref, "n=%d" % P.shape[0])
