"""GPU parity: the HIP path (through the C ABI) against the CPU oracle.

Bar: bit-exact indices and bit-exact FP32 squared distances, on every
configuration, for every voxel resolution, tile size and workgroup count
(all output-neutral by construction).  Full workload sizes are covered here
for the room (80,000 -> 20,000) and the LiDAR multi-stage run
(114,624 -> 28,656 -> 7,164 -> 1,791); the 1M-point cloud is covered in
test_gpu_large.py.
"""
import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu


def rf():
    import paper_2606_06255_amd as m
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU")
    return m


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).cuda()


def host(t):
    return t.cpu().numpy()


def assert_same(got, ref, what=""):
    gi, gd = host(got[0]), host(got[1])
    ri, rd = ref
    bad = np.flatnonzero(gi != ri)
    assert bad.size == 0, "%s: first index mismatch at %d: %d vs %d" % (what, bad[0], gi[bad[0]], ri[bad[0]])
    bd = np.flatnonzero(gd.view(np.uint32) != rd.view(np.uint32))
    assert bd.size == 0, "%s: first d2 mismatch at %d: %r vs %r" % (what, bd[0], gd[bd[0]], rd[bd[0]])


def test_plain_cube(oracle_lib):
    m = rf()
    for seed in (0, 1):
        P = synth.cube(seed)
        ref = oracle_lib.fps(P, 1024, 0)
        x = dev(P)
        assert_same(m.fps_plain(x, 1024, 0, variant=1), ref, "1wg")
        for g in (0, 1, 2, 7):
            assert_same(m.fps_plain(x, 1024, 0, variant=0, groups=g), ref, "persistent g=%d" % g)


def test_rfps_cube_partitions(oracle_lib):
    m = rf()
    P = synth.cube(0)
    ref = oracle_lib.fps(P, 1024, 0)
    x = dev(P)
    for n_vox in (1, 4, 8, 16, 32):
        for tile in (0, 1, 7):
            idx = m.build_index(x, n_vox=n_vox, tile=tile)
            for g in (1, 3, 64, 0):
                for la, fl in ((0, 0), (3, 0), (4, 0), (8, 0), (0, m.F_SINGLE_PICK)):
                    got = m.sample(idx, 1024, 0, groups=g, lookahead=la, flags=fl)
                    st = m.read_status(idx)
                    what = "n_vox=%d tile=%d g=%d lookahead=%d flags=%d" % (n_vox, tile, g, la, fl)
                    if st == 6:
                        # only a single workgroup can run out of LDS on 4096 points;
                        # the error is clean: every output is poisoned
                        assert g == 1, what
                        assert np.all(host(got[0]) == -1)
                        continue
                    assert st == 0, (what, st)
                    assert_same(got, ref, what)


def test_rfps_flags_cube(oracle_lib):
    m = rf()
    P = synth.cube(3)
    ref = oracle_lib.fps(P, 1024, 5)
    idx = m.build_index(dev(P), n_vox=8)
    for flags in (m.F_NO_PRUNE, m.F_NO_POINT_SKIP, m.F_TELEMETRY, m.F_TRACE,
                  m.F_NO_PRUNE | m.F_NO_POINT_SKIP, m.F_SINGLE_PICK, m.F_SINGLE_PICK | m.F_NO_POINT_SKIP):
        assert_same(m.sample(idx, 1024, 5, flags=flags), ref, "flags=%d" % flags)


def test_index_shape_matches_cpu_grid(oracle_lib):
    m = rf()
    for P, n_vox in ((synth.cube(0), 16), (synth.room(0), 24), (synth.lidar(0)[::3], 64)):
        pmin, L, vid = oracle_lib.voxelize(P, n_vox)
        idx = m.build_index(dev(P), n_vox=n_vox, tile=64)
        info = m.read_index_info(idx)
        u, c = np.unique(vid, return_counts=True)
        assert info["n_voxels"] == len(u)
        assert info["n_tiles"] == int(np.sum((c + 63) // 64))
        assert info["voxel_edge"] == L
        assert info["pmin"] == list(pmin)


def test_room_full(oracle_lib):
    m = rf()
    P = synth.room(0)
    ref = oracle_lib.fps(P, 20000, 0, threads=0)
    x = dev(P)
    assert_same(m.fps(x, 20000, 0), ref, "rfps default")
    assert_same(m.fps(x, 20000, 0, n_vox=48, tile=32, groups=128), ref, "rfps n48 t32 g128")
    assert_same(m.fps(x, 20000, 0, groups=32, lookahead=8), ref, "rfps g32 lookahead 8")
    assert_same(m.fps(x, 20000, 0, groups=256, lookahead=2), ref, "rfps g256 lookahead 2")
    assert_same(m.fps(x, 20000, 0, groups=256, lookahead=3), ref, "rfps g256 lookahead 3")
    assert_same(m.fps(x, 20000, 0, groups=256, lookahead=4), ref, "rfps g256 lookahead 4")
    assert_same(m.fps(x, 20000, 0, flags=m.F_SINGLE_PICK), ref, "rfps single pick")
    assert_same(m.fps_plain(x, 20000, 0, variant=0), ref, "plain persistent")


def test_range_shells(oracle_lib):
    # range shells only change the partition: the result must not move
    m = rf()
    cases = ((synth.cube(2), 1024, (0.05, 0.3)), (synth.room(0), 20000, (1.0, 3.0)),
             (synth.lidar(1), 28656, (5.0, 20.0)))
    for P, M, spacings in cases:
        ref = oracle_lib.fps(P, M, 0, threads=0)
        x = dev(P)
        for sh in spacings:
            for n_vox in (8, 32, 128):
                idx = m.build_index(x, n_vox=n_vox, shell=sh)
                assert idx.handle.shells > 1
                got = m.sample(idx, M, 0)
                assert m.read_status(idx) == 0
                assert_same(got, ref, "N=%d shell=%g n_vox=%d" % (P.shape[0], sh, n_vox))
    # shells of growing cells coarsen the sparse far range of a spinning sensor
    P = synth.lidar(1)
    flat = m.read_index_info(m.build_index(dev(P), n_vox=96))["n_tiles"]
    shelled = m.read_index_info(m.build_index(dev(P), n_vox=96, shell=10.0))["n_tiles"]
    assert shelled < flat


def test_lidar_multistage(oracle_lib):
    # every stage samples the previous stage's picks in pick order; on the
    # device the next input comes from rfps_gather_xyz
    m = rf()
    P = synth.lidar(0)
    sizes = synth.lidar_stage_sizes(P.shape[0])
    cur, x = P, dev(P)
    for k, mm in enumerate(sizes[1:]):
        ref = oracle_lib.fps(cur, mm, 0, threads=0)
        got = m.fps(x, mm, 0)
        assert_same(got, ref, "stage %d" % (k + 1))
        cur = cur[ref[0]]
        x = m.gather_xyz(x, got[0])
        assert np.array_equal(host(x).view(np.uint32), cur.view(np.uint32))


def test_gather_out_of_range():
    m = rf()
    P = synth.cube(4)[:100]
    idx = torch.tensor([5, -1, 99, 100, 0], dtype=torch.int32, device="cuda:0")
    got = host(m.gather_xyz(dev(P), idx))
    assert np.array_equal(got[[0, 2, 4]], P[[5, 99, 0]])
    assert np.all(np.isnan(got[[1, 3]]))
    # NaN input is then reported by the next build
    idx2 = m.build_index(dev(np.ascontiguousarray(got)))
    assert m.read_status(idx2) == 2


def test_edge_cases(oracle_lib):
    m = rf()
    rng = np.random.default_rng(11)
    cases = [
        ("n1", np.zeros((1, 3), np.float32), 1, 0),
        ("m1", synth.cube(0)[:500], 1, 17),
        ("m_eq_n", synth.cube(1)[:300], 300, 299),
        ("identical", np.ones((1000, 3), np.float32), 50, 3),
        ("duplicates", np.repeat(synth.cube(2)[:200], 5, axis=0), 600, 0),
        ("lattice_ties", np.stack(np.meshgrid(*[np.arange(10)] * 3, indexing="ij"), -1)
         .reshape(-1, 3).astype(np.float32), 1000, 0),
        ("ragged_4097", rng.random((4097, 3), dtype=np.float32), 4097, 4096),
        ("ragged_10007", rng.normal(size=(10007, 3)).astype(np.float32), 3001, 5),
        ("planar", np.c_[rng.random((5000, 2)), np.zeros(5000)].astype(np.float32), 2000, 0),
        ("wide_range", (rng.normal(size=(3000, 3)) * 1e4).astype(np.float32), 1500, 0),
        ("tiny_scale", (rng.random((3000, 3)) * 1e-6).astype(np.float32), 1500, 0),
    ]
    for name, P, mm, s in cases:
        ref = oracle_lib.fps(P, mm, s)
        x = dev(P)
        for n_vox in (1, 8, 64):
            assert_same(m.fps(x, mm, s, n_vox=n_vox), ref, "%s n_vox=%d" % (name, n_vox))
        assert_same(m.fps(x, mm, s, groups=7, lookahead=2), ref, name + " g7 la2")
        assert_same(m.fps(x, mm, s, groups=64, lookahead=4), ref, name + " g64 la4")
        assert_same(m.fps(x, mm, s, flags=m.F_SINGLE_PICK), ref, name + " single")
        assert_same(m.fps(x, mm, s, flags=m.F_UNFUSED), ref, name + " unfused")
        assert_same(m.fps_plain(x, mm, s, variant=0), ref, name + " plain0")
        assert_same(m.fps_plain(x, mm, s, variant=1), ref, name + " plain1")


def test_repeatable(oracle_lib):
    m = rf()
    P = synth.room(1)[:30000]
    ref = oracle_lib.fps(P, 7000, 0, threads=0)
    idx = m.build_index(dev(P))
    for _ in range(3):
        assert_same(m.sample(idx, 7000, 0), ref, "repeat")


def test_nonfinite_input_reports_and_poisons():
    m = rf()
    P = synth.cube(0).copy()
    P[123, 2] = np.nan
    x = dev(P)
    idx = m.build_index(x)
    oi, od = m.sample(idx, 64, 0)
    assert m.read_status(idx) == 2
    assert np.all(host(oi) == -1) and np.all(np.isnan(host(od)))
    oi, od = m.sample(idx, 64, 0, flags=m.F_UNFUSED)
    assert m.read_status(idx) == 2
    assert np.all(host(oi) == -1) and np.all(np.isnan(host(od)))
    with pytest.raises(m.RfpsError) as e:
        m.fps_plain(x, 64, 0, variant=0)
    assert e.value.status == 2


def test_capacity_error_when_one_group_is_too_small():
    m = rf()
    P = synth.room(0)
    idx = m.build_index(dev(P))
    oi, od = m.sample(idx, 100, 0, groups=1)
    assert m.read_status(idx) == 6
    assert np.all(host(oi) == -1)


def test_host_errors():
    m = rf()
    x = dev(synth.cube(0))
    idx = m.build_index(x)
    with pytest.raises(m.RfpsError):
        m.sample(idx, 5000, 0)
    with pytest.raises(m.RfpsError):
        m.sample(idx, 10, 4096)
    with pytest.raises(ValueError):
        m.build_index(x.double())


def test_telemetry_sane(oracle_lib):
    m = rf()
    P = synth.room(2)[:20000]
    idx = m.build_index(dev(P), n_vox=24)
    info = m.read_index_info(idx)
    # strict decreases are a property of the sequence, not of the partition
    _, _, cpu = oracle_lib.rfps_cpu(P, 5000, 0, n_vox=24)
    for fl in (m.F_TELEMETRY | m.F_SINGLE_PICK, m.F_TELEMETRY):
        m.sample(idx, 5000, 0, flags=fl)
        t = m.read_telemetry(idx)
        assert t["iters"] == 4998 and t["tiles"] == info["n_tiles"]
        assert 0 < t["tiles_pruned"] < t["tile_tests"]
        assert t["points_updated"] <= t["points_visited"] - t["points_skipped"]
        if fl & m.F_SINGLE_PICK:
            assert t["tile_tests"] == t["iters"] * t["tiles"]
            assert t["exchanges"] == 4999
            # one strict decrease per (point, selection), as in plain FPS
            assert t["points_updated"] == cpu["points_updated"]
        else:
            assert 0 < t["exchanges"] < 4999
            # a round applies all its selections at once: a point lowered by
            # several of them is stored (and counted) once
            assert 0 < t["points_updated"] <= cpu["points_updated"]
            assert t["tick_hz"] > 0 and t["ticks_merge"] > 0 and t["ticks_exchange"] > 0


def test_trace_records_every_exchange():
    m = rf()
    idx = m.build_index(dev(synth.cube(0)))
    m.sample(idx, 1024, 0, flags=m.F_TRACE | m.F_SINGLE_PICK)
    tr, hz = m.read_trace(idx)
    assert tr.shape == (1023, 2) and hz > 0
    assert np.all(tr[:, 1] >= tr[:, 0])
    m.sample(idx, 1024, 0, flags=m.F_TRACE)
    tr, hz = m.read_trace(idx)
    picks = (tr[:, 1] >> np.uint64(48)).astype(np.int64)
    assert picks.sum() == 1023 and np.all(picks >= 1)
    t1 = tr[:, 1] & np.uint64((1 << 48) - 1)
    assert np.all(t1 >= tr[:, 0])


def test_unfused_cube_and_room(oracle_lib):
    # the per-iteration-launch sampler: every selection is its own pair of
    # launches, with the state in device memory between them
    m = rf()
    P = synth.cube(4)
    ref = oracle_lib.fps(P, 1024, 9)
    ref_eu = oracle_lib.fps(P, 1024, 9, euclid=True)
    x = dev(P)
    for n_vox in (1, 4, 16):
        for tile in (0, 1, 7):
            idx = m.build_index(x, n_vox=n_vox, tile=tile)
            for fl in (0, m.F_NO_PRUNE, m.F_NO_POINT_SKIP, m.F_NO_PRUNE | m.F_NO_POINT_SKIP):
                what = "unfused n_vox=%d tile=%d flags=%d" % (n_vox, tile, fl)
                assert_same(m.sample(idx, 1024, 9, flags=m.F_UNFUSED | fl), ref, what)
                assert m.read_status(idx) == 0, what
            assert_same(m.sample(idx, 1024, 9, flags=m.F_UNFUSED | m.F_SQRT), ref_eu, "unfused euclid")
    R = synth.room(0)
    ref = oracle_lib.fps(R, 20000, 0, threads=0)
    xr = dev(R)
    assert_same(m.fps(xr, 20000, 0, flags=m.F_UNFUSED), ref, "unfused room")
    # the persistent samplers still work on an index the unfused one used
    idx = m.build_index(xr)
    assert_same(m.sample(idx, 20000, 0, flags=m.F_UNFUSED), ref, "unfused room, reused index")
    assert_same(m.sample(idx, 20000, 0), ref, "multi-pick after unfused")
    with pytest.raises(m.RfpsError) as e:
        m.sample(idx, 100, 0, flags=m.F_UNFUSED | m.F_TELEMETRY)
    assert e.value.status == 5
