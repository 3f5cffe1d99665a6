"""Batched sampling (rfps_sample_batched) against the CPU oracle, cloud by
cloud: many clouds of uneven size in one persistent launch must give, for
every cloud, exactly the FPS sequence of that cloud alone (indices local to
the cloud, FP32 squared distances bit for bit)."""
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


def _concat(clouds):
    sizes = [c.shape[0] for c in clouds]
    offsets = np.zeros(len(clouds) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    return np.ascontiguousarray(np.concatenate(clouds, axis=0).astype(np.float32)), offsets


def _expect(xyz, offsets, m, starts):
    idx, d2 = [], []
    for c in range(len(m)):
        pts = xyz[offsets[c]:offsets[c + 1]]
        threads = oracle.num_threads() if pts.shape[0] > 20000 else 1
        i, d = oracle.fps(pts, int(m[c]), int(starts[c]) if starts is not None else 0, threads=threads)
        idx.append(i)
        d2.append(d)
    return np.concatenate(idx), np.concatenate(d2)


def _check(rf, xyz, offsets, m, starts=None, **kw):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    idx, d2 = rf.sample_batched(x, offsets, m, starts, **kw)
    torch.cuda.synchronize()
    ei, ed = _expect(xyz, offsets, m, starts)
    gi, gd = idx.cpu().numpy(), d2.cpu().numpy()
    assert np.array_equal(gi, ei), "indices differ (%s)" % (kw,)
    assert np.array_equal(gd.view(np.uint32), ed.view(np.uint32)), "distances differ (%s)" % (kw,)


def _small_batch(seed):
    rng = np.random.default_rng(seed)
    clouds = [synth.cube(seed, 500), synth.cube(seed + 1, 1), synth.cube(seed + 2, 3000),
              synth.room(seed, n=2000), synth.cube(seed + 3, 7), synth.lidar(seed, beams=16, azimuth_steps=90,
                                                                             n_out=1400)]
    xyz, offsets = _concat(clouds)
    sizes = np.diff(offsets)
    m = np.array([125, 1, 3000, 500, 7, 350], dtype=np.int32)
    starts = np.array([rng.integers(0, s) for s in sizes], dtype=np.int32)
    return xyz, offsets, m, starts


@pytest.mark.parametrize("groups", [0, 2, 4, 8, 16])
@pytest.mark.parametrize("lookahead", [2, 3, 4, 8])
def test_small_batch_partitions(rf, groups, lookahead):
    xyz, offsets, m, starts = _small_batch(3)
    _check(rf, xyz, offsets, m, starts, groups=groups, lookahead=lookahead)


@pytest.mark.parametrize("n_vox,tile,shell", [(0, 64, 0.0), (0, 16, 0.0), (8, 64, 0.0), (32, 7, 0.0),
                                              (1, 64, 0.0), (0, 64, 0.4), (24, 32, 2.0)])
def test_small_batch_grids(rf, n_vox, tile, shell):
    xyz, offsets, m, starts = _small_batch(5)
    _check(rf, xyz, offsets, m, starts, n_vox=n_vox, tile=tile, shell=shell)
    _check(rf, xyz, offsets, m, None, n_vox=n_vox, tile=tile, flags=rf.F_NO_POINT_SKIP, shell=shell)


def test_uneven_batch_full(rf):
    # the uneven room / LiDAR mix at full per-cloud sizes, 8 clouds
    xyz, offsets, m = synth.batch(seed=1, b=8)
    _check(rf, xyz, offsets, m)


def test_many_tiny_clouds(rf):
    clouds = [synth.cube(s, 1 + (s * 37) % 200) for s in range(300)]
    xyz, offsets = _concat(clouds)
    sizes = np.diff(offsets)
    m = np.maximum(1, sizes // 3).astype(np.int32)
    _check(rf, xyz, offsets, m, groups=4)


def test_duplicates_and_degenerate(rf):
    same = np.ones((300, 3), dtype=np.float32)
    line = np.zeros((65, 3), dtype=np.float32)
    line[:, 0] = np.arange(65, dtype=np.float32)
    xyz, offsets = _concat([same, line, synth.cube(0, 100)])
    _check(rf, xyz, offsets, np.array([300, 65, 100], dtype=np.int32))


def test_device_side_errors(rf):
    dev = torch.device("cuda:0")
    xyz, offsets, m, _ = _small_batch(7)
    x = torch.from_numpy(xyz).to(dev)
    ws = rf.BatchWorkspace(xyz.shape[0], len(m), dev)
    # m_total that disagrees with sum(m)
    idx, _ = rf.sample_batched(x, offsets, m, m_total=int(m.sum()) - 1, ws=ws, check=False)
    assert rf.batched_read_status(ws) == 1
    assert (idx.cpu() == -1).all()
    # m larger than its cloud
    bad_m = m.copy()
    bad_m[0] = offsets[1] + 1
    idx, _ = rf.sample_batched(x, offsets, bad_m, ws=ws, check=False)
    assert rf.batched_read_status(ws) == 1
    assert (idx.cpu() == -1).all()
    # offsets that do not end at n
    bad_off = offsets.copy()
    bad_off[-1] -= 1
    rf.sample_batched(x, bad_off, m, ws=ws, check=False)
    assert rf.batched_read_status(ws) == 1
    # a start outside its cloud
    starts = np.zeros(len(m), dtype=np.int32)
    starts[2] = offsets[3] - offsets[2]
    rf.sample_batched(x, offsets, m, starts, ws=ws, check=False)
    assert rf.batched_read_status(ws) == 1
    # a non-finite coordinate in one cloud poisons the whole call
    y = x.clone()
    y[offsets[3] + 5, 1] = float("nan")
    idx, d2 = rf.sample_batched(y, offsets, m, ws=ws, check=False)
    assert rf.batched_read_status(ws) == 2
    assert (idx.cpu() == -1).all() and torch.isnan(d2.cpu()).all()
    # and the same workspace then works again
    idx, _ = rf.sample_batched(x, offsets, m, ws=ws)
    ei, _ = _expect(xyz, offsets, m, None)
    assert np.array_equal(idx.cpu().numpy(), ei)


def test_capacity_is_reported(rf):
    # one 120k-point cloud cannot be held by a team of 2 workgroups
    xyz = synth.room(0, n=120000)
    dev = torch.device("cuda:0")
    offsets = np.array([0, xyz.shape[0]], dtype=np.int32)
    idx, _ = rf.sample_batched(torch.from_numpy(xyz).to(dev), offsets, [100], groups=2, check=False)
    with pytest.raises(rf.RfpsError) as e:
        rf.sample_batched(torch.from_numpy(xyz).to(dev), offsets, [100], groups=2)
    assert e.value.status == 6
    assert (idx.cpu() == -1).all()


def test_telemetry(rf):
    dev = torch.device("cuda:0")
    xyz, offsets, m, starts = _small_batch(11)
    ws = rf.BatchWorkspace(xyz.shape[0], len(m), dev)
    rf.sample_batched(torch.from_numpy(xyz).to(dev), offsets, m, starts, ws=ws, flags=rf.F_TELEMETRY)
    t = rf.batched_read_telemetry(ws)
    assert t["iters"] == int(np.maximum(m - 2, 0).sum())
    assert 0 < t["exchanges"] <= int((m - 1).sum())
    assert t["tiles_pruned"] <= t["tile_tests"]
    assert 0 < t["points_updated"] <= t["points_visited"]


def test_graph_capture_replays(rf):
    dev = torch.device("cuda:0")
    xyz, offsets, m = synth.batch(seed=2, b=6, n_hi=30000)
    x = torch.from_numpy(xyz).to(dev)
    off_d = torch.from_numpy(offsets).to(dev)
    m_d = torch.from_numpy(m).to(dev)
    mt = int(m.sum())
    ws = rf.BatchWorkspace(xyz.shape[0], len(m), dev)
    ref_i, ref_d = rf.sample_batched(x, off_d, m_d, m_total=mt, ws=ws)
    ref_i, ref_d = ref_i.clone(), ref_d.clone()
    out_i = torch.full((mt,), -7, dtype=torch.int32, device=dev)
    out_d = torch.zeros(mt, dtype=torch.float32, device=dev)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        rf.sample_batched(x, off_d, m_d, m_total=mt, ws=ws, out_idx=out_i, out_d2=out_d)  # warm-up
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        rf.sample_batched(x, off_d, m_d, m_total=mt, ws=ws, out_idx=out_i, out_d2=out_d, check=False)
    for rep in range(3):
        out_i.fill_(-7)
        out_d.zero_()
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert rf.batched_read_status(ws) == 0, rep
        assert torch.equal(out_i, ref_i), rep
        assert torch.equal(out_d.view(torch.int32), ref_d.view(torch.int32)), rep
        # eager work on the same workspace between replays
        rf.sample_batched(x, off_d, m_d, m_total=mt, ws=ws, groups=8)
    ei, _ = _expect(xyz, offsets, m, None)
    assert np.array_equal(ref_i.cpu().numpy(), ei)


def test_autotuner_keeps_result(rf):
    dev = torch.device("cuda:0")
    xyz, offsets, m = synth.batch(seed=4, b=5, n_hi=40000)
    chosen, ms, (idx, d2) = rf.autotune_batched(torch.from_numpy(xyz).to(dev), offsets, m, reps=1)
    assert ms > 0
    assert chosen["groups"] in (4, 8, 16, 32) and chosen["lookahead"] in (2, 3, 4, 8) and chosen["tile"] in (32, 64)
    ei, ed = _expect(xyz, offsets, m, None)
    assert np.array_equal(idx.cpu().numpy(), ei)
    assert np.array_equal(d2.cpu().numpy().view(np.uint32), ed.view(np.uint32))
