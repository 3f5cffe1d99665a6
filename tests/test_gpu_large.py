"""Full-size parity: the 1M-point dense LiDAR-like cloud (1,048,576 -> 65,536)
and the uneven batch of 32 clouds, in the launch configurations the benchmark
times, against the whole oracle sequence (every index and every FP32
distance), in both the squared and the Euclidean distance form; and the
largest clouds one launch holds on chip: a 1.24M-point LiDAR-like sweep at
the default grid, and a 1.05M-point room-like cloud, whose default grid does
not fit, through the coarser-grid fallback."""
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


@pytest.fixture(scope="module")
def dense():
    return synth.dense_lidar(0)


def _same(got, ref, what):
    gi, gd = got[0].cpu().numpy(), got[1].cpu().numpy()
    ri, rd = ref
    bad = np.flatnonzero(gi != ri)
    assert bad.size == 0, "%s: first index mismatch at %d of %d" % (what, bad[0], len(ri))
    bd = np.flatnonzero(gd.view(np.uint32) != rd.view(np.uint32))
    assert bd.size == 0, "%s: first distance mismatch at %d: %r vs %r" % (what, bd[0], gd[bd[0]], rd[bd[0]])


@pytest.mark.parametrize("euclid", [False, True])
def test_dense_lidar_full(rf, dense, euclid):
    m = 65536
    print("dense 1M -> 65536, euclid=%s" % euclid, flush=True)
    ref = oracle.fps(dense, m, 0, threads=0, euclid=euclid)
    x = torch.from_numpy(dense).cuda()
    flags = rf.F_SQRT if euclid else 0
    _same(rf.fps(x, m, 0, flags=flags), ref, "default launch")
    if not euclid:
        _same(rf.fps(x, m, 0, lookahead=4), ref, "lookahead 4")


@pytest.mark.parametrize("euclid", [False, True])
def test_batch32_full(rf, euclid):
    xyz, offsets, m = synth.batch(0, b=32)
    print("batch of 32, sum N %d, sum M %d, euclid=%s" % (xyz.shape[0], int(m.sum()), euclid), flush=True)
    ei, ed = [], []
    for c in range(len(m)):
        i, d = oracle.fps(xyz[offsets[c]:offsets[c + 1]], int(m[c]), 0, threads=0, euclid=euclid)
        ei.append(i)
        ed.append(d)
    ref = (np.concatenate(ei), np.concatenate(ed))
    x = torch.from_numpy(xyz).cuda()
    flags = rf.F_SQRT if euclid else 0
    _same(rf.sample_batched(x, offsets, m, flags=flags), ref, "default launch")
    # (fewer than 32 workgroups per cloud cannot hold the 100k-point clouds
    # on chip: that configuration reports RFPS_ERR_CAPACITY)
    _same(rf.sample_batched(x, offsets, m, lookahead=4, flags=flags), ref, "lookahead 4")


def test_largest_lidar_cloud(rf):
    # 128 beams x 9,700 azimuth steps: the largest workgroup share is about
    # 152 KB of the 156.9 KB the default launch has; 10,000 steps (161 KB)
    # report RFPS_ERR_CAPACITY
    P = synth.lidar(1, beams=128, azimuth_steps=9700, drop=0)
    n, m = P.shape[0], P.shape[0] // 16
    print("largest LiDAR-like cloud %d -> %d" % (n, m), flush=True)
    ref = oracle.fps(P, m, 0, threads=0)
    x = torch.from_numpy(P).cuda()
    idx = rf.build_index(x)
    info = rf.read_index_info(idx)
    print("n_vox %d, %d tiles, %.1f points per tile" % (idx.n_vox, info["n_tiles"], n / info["n_tiles"]), flush=True)
    got = rf.sample(idx, m, 0)
    rf._check(rf.read_status(idx), "device status")
    _same(got, ref, "1.24M LiDAR")


def test_room_past_default_grid_falls_back(rf):
    from paper_2606_06255_amd import param_model

    class DefaultRule:
        """Chooses what the default rule chooses, so that the fallback runs."""
        def choose(self, x):
            return rf.default_n_vox(x.shape[0]), 0.0, 0, None

    # at the default 192 bins (about 6 points per tile) the largest workgroup
    # share would be about 162 KB of 156.9 KB; 128 bins, the next grid the
    # fallback tries, need about 147 KB
    P = synth.room(1, n=1_050_000)
    n, m = P.shape[0], 50_000
    print("room-like cloud %d -> %d, default n_vox %d" % (n, m, rf.default_n_vox(n)), flush=True)
    x = torch.from_numpy(P).cuda()
    with pytest.raises(rf.RfpsError) as e:
        rf.fps(x, m, 0)
    assert e.value.status == 6
    ref = oracle.fps(P, m, 0, threads=0)
    i, d, (nv, sh) = param_model.fps_auto(DefaultRule(), x, m, 0)
    print("fell back to n_vox %d" % nv, flush=True)
    assert nv < rf.default_n_vox(n)
    _same((i, d), ref, "1.05M room, fallback grid")
