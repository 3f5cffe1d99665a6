"""rfps_sample_batched_noalloc (the batched call on the library's fixed
scratch array, for callers that cannot allocate) against rfps_sample_batched
on the same inputs: indices and FP32 distance bits must be identical, on two
calls in a row (the second one smaller, so it runs on whatever the first left
in the array), with the larger batch also checked against the oracle."""
import sys

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


def _batch(seed, sizes):
    rng = np.random.default_rng(seed)
    clouds = []
    for k, n in enumerate(sizes):
        if k % 3 == 0:
            clouds.append(synth.room(seed + k, n=n))
        elif k % 3 == 1:
            clouds.append(synth.cube(seed + k, n))
        else:
            clouds.append(synth.lidar(seed + k, beams=16, azimuth_steps=max(1, -(-n // 16) + 8), n_out=n))
    xyz = np.ascontiguousarray(np.concatenate(clouds, axis=0).astype(np.float32))
    offsets = np.zeros(len(sizes) + 1, dtype=np.int32)
    offsets[1:] = np.cumsum(sizes)
    m = np.array([max(1, n // 4) for n in sizes], dtype=np.int32)
    starts = np.array([rng.integers(0, n) for n in sizes], dtype=np.int32)
    return xyz, offsets, m, starts


def _run_both(rf, xyz, offsets, m, starts, **kw):
    dev = torch.device("cuda:0")
    x = torch.from_numpy(xyz).to(dev)
    off_d = torch.from_numpy(offsets).to(dev)
    m_d = torch.from_numpy(m).to(dev)
    st_d = torch.from_numpy(starts).to(dev)
    mt = int(m.sum())
    ri, rd = rf.sample_batched(x, off_d, m_d, st_d, m_total=mt, **kw)
    # poisoned outputs must be overwritten by the call
    ni = torch.full((mt,), -7, dtype=torch.int32, device=dev)
    nd = torch.full((mt,), float("nan"), dtype=torch.float32, device=dev)
    print("noalloc: batch=%d n=%d m_total=%d %s" % (len(m), xyz.shape[0], mt, kw), flush=True)
    rf.sample_batched_noalloc(x, off_d, m_d, mt, ni, nd, starts=st_d, **kw)
    torch.cuda.synchronize()
    return ri.cpu().numpy(), rd.cpu().numpy(), ni.cpu().numpy(), nd.cpu().numpy()


def _same(a_i, a_d, b_i, b_d):
    assert np.array_equal(a_i, b_i), "indices differ"
    assert np.array_equal(a_d.view(np.uint32), b_d.view(np.uint32)), "distances differ"


def test_noalloc_matches_workspace_call_twice(rf):
    big = _batch(11, [9000, 3000, 15000, 1, 700, 12000, 5000, 64])
    small = _batch(12, [2500, 40, 6000])
    for xyz, offsets, m, starts in (big, small):
        ri, rd, ni, nd = _run_both(rf, xyz, offsets, m, starts)
        _same(ri, rd, ni, nd)
    # the first (larger) batch against the oracle, cloud by cloud
    xyz, offsets, m, starts = big
    ri, rd, ni, nd = _run_both(rf, xyz, offsets, m, starts)
    _same(ri, rd, ni, nd)
    o = 0
    for c in range(len(m)):
        ei, ed = oracle.fps(xyz[offsets[c]:offsets[c + 1]], int(m[c]), int(starts[c]))
        _same(ni[o:o + m[c]], nd[o:o + m[c]], ei, ed)
        o += int(m[c])


def test_noalloc_options_and_limit(rf):
    xyz, offsets, m, starts = _batch(13, [4000, 800, 2500])
    for kw in ({"groups": 4, "lookahead": 4}, {"n_vox": 16, "tile": 32}, {"flags": rf.F_SQRT}):
        ri, rd, ni, nd = _run_both(rf, xyz, offsets, m, starts, **kw)
        _same(ri, rd, ni, nd)
    # beyond the fixed array: a clear error, nothing enqueued
    n = 1 << 26
    assert rf.lib().rfps_batched_workspace_size(n, 1, None) > rf.noalloc_scratch_bytes()
    dev = torch.device("cuda:0")
    dummy = torch.zeros(4, dtype=torch.int32, device=dev)
    st = rf.lib().rfps_sample_batched_noalloc(dummy.data_ptr(), n, dummy.data_ptr(), dummy.data_ptr(), None, 1, 1,
                                              None, dummy.data_ptr(), None, None)
    assert st == 9 and rf.STATUS_NAMES[st] == "RFPS_ERR_SCRATCH_LIMIT"
    print("noalloc limit ok", file=sys.stderr, flush=True)
