"""Seeded random configurations of every sampler option against the oracle.

Each case draws a cloud shape (uniform, clustered, planar, on a line, on a
coarse grid with many equal distances, with duplicates, wide dynamic range),
its size and sample count, and a launch configuration (voxel bins, tile size,
workgroups, lookahead, one-pick / unfused / no-prune / no-skip, squared or
Euclidean distances), and compares indices and distances bit for bit.  The
seeds are fixed, so every run checks the same cases."""
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


def cloud(rng, n):
    kind = int(rng.integers(0, 7))
    if kind == 0:
        P = rng.random((n, 3))
    elif kind == 1:
        c = rng.normal(size=(int(rng.integers(1, 9)), 3)) * 10
        P = c[rng.integers(0, len(c), n)] + rng.normal(size=(n, 3)) * 0.1
    elif kind == 2:
        P = np.c_[rng.random((n, 2)) * 5, np.full(n, 0.25)]
    elif kind == 3:
        t = rng.random(n)
        P = np.c_[t, 2 * t, -t] + rng.normal(size=(n, 3)) * 1e-3
    elif kind == 4:
        P = rng.integers(-12, 13, size=(n, 3)) * 0.1
    elif kind == 5:
        base = rng.random((max(1, n // 4), 3))
        P = base[rng.integers(0, len(base), n)]
    else:
        P = rng.normal(size=(n, 3)) * 10.0 ** rng.integers(-3, 5)
    return np.ascontiguousarray(P.astype(np.float32)), kind


def same(got, ref, what):
    gi, gd = got[0].cpu().numpy(), got[1].cpu().numpy()
    ri, rd = ref
    bad = np.flatnonzero(gi != ri)
    assert bad.size == 0, "%s: first index mismatch at %d" % (what, bad[0])
    bd = np.flatnonzero(gd.view(np.uint32) != rd.view(np.uint32))
    assert bd.size == 0, "%s: first distance mismatch at %d" % (what, bd[0])


@pytest.mark.parametrize("seed", range(20))
def test_random_single_cloud(rf, seed):
    rng = np.random.default_rng(1000 + seed)
    for case in range(8):
        n = int(np.exp(rng.uniform(np.log(2), np.log(30000))))
        P, kind = cloud(rng, n)
        m = int(rng.integers(1, n + 1)) if n < 3000 else int(rng.integers(1, n // 2))
        start = int(rng.integers(0, n))
        euclid = bool(rng.integers(0, 4) == 0)
        mode = ("multi", "single", "unfused", "noprune")[int(rng.integers(0, 4))]
        flags = {"multi": 0, "single": rf.F_SINGLE_PICK, "unfused": rf.F_UNFUSED, "noprune": rf.F_NO_PRUNE}[mode]
        if rng.integers(0, 3) == 0:
            flags |= rf.F_NO_POINT_SKIP
        if euclid:
            flags |= rf.F_SQRT
        n_vox = int(rng.choice([0, 1, 2, 5, 16, 40, 128]))
        tile = int(rng.choice([0, 1, 3, 16, 33, 64]))
        groups = int(rng.choice([0, 0, 2, 7, 32, 64, 128, 256]))
        la = int(rng.choice([0, 2, 3, 4, 8]))
        what = "seed %d case %d: kind %d n %d m %d start %d mode %s flags %d n_vox %d tile %d groups %d la %d" % (
            seed, case, kind, n, m, start, mode, flags, n_vox, tile, groups, la)
        print(what, flush=True)
        ref = oracle.fps(P, m, start, threads=0, euclid=euclid)
        idx = rf.build_index(torch.from_numpy(P).cuda(), n_vox=n_vox, tile=tile)
        got = rf.sample(idx, m, start, groups=groups, lookahead=la, flags=flags)
        st = rf.read_status(idx)
        if st == 6:
            # a share of the cloud too large for one workgroup's LDS is a clean error
            assert np.all(got[0].cpu().numpy() == -1), what
            continue
        assert st == 0, (what, st)
        same(got, ref, what)


@pytest.mark.parametrize("seed", range(8))
def test_random_batches(rf, seed):
    rng = np.random.default_rng(2000 + seed)
    B = int(rng.integers(1, 24))
    clouds, ms, starts = [], [], []
    for _ in range(B):
        n = int(np.exp(rng.uniform(0, np.log(12000))))
        P, _ = cloud(rng, n)
        clouds.append(P)
        ms.append(int(rng.integers(1, n + 1)))
        starts.append(int(rng.integers(0, n)))
    euclid = bool(rng.integers(0, 2))
    offsets = np.zeros(B + 1, dtype=np.int32)
    offsets[1:] = np.cumsum([c.shape[0] for c in clouds])
    xyz = np.ascontiguousarray(np.concatenate(clouds))
    m = np.array(ms, dtype=np.int32)
    st = np.array(starts, dtype=np.int32)
    ei, ed = [], []
    for c in range(B):
        i, d = oracle.fps(clouds[c], ms[c], starts[c], euclid=euclid)
        ei.append(i)
        ed.append(d)
    la = int(rng.choice([0, 2, 3, 4, 8]))
    groups = int(rng.choice([0, 2, 4, 8, 16]))
    what = "seed %d: %d clouds, sum N %d, euclid %s, groups %d, la %d" % (seed, B, xyz.shape[0], euclid, groups, la)
    print(what, flush=True)
    try:
        got = rf.sample_batched(torch.from_numpy(xyz).cuda(), offsets, m, st, groups=groups, lookahead=la,
                                flags=rf.F_SQRT if euclid else 0)
    except rf.RfpsError as e:
        # too few workgroups per cloud for the largest cloud's share of LDS
        assert e.status == 6, (what, e.status)
        return
    same(got, (np.concatenate(ei), np.concatenate(ed)), what)
