"""What the trained voxel-parameter network gains over the default rule.

The clouds are fresh: drawn with a seed the sweep never used, at sizes over
the whole training range, both kinds of scene.  On each, the network's grid
and the default rule's grid are timed (build + sample, median of repeated
runs on the same stream) and must give the same sequence, whose prefix must
be the oracle's.  The network must gain at least 5 % in the geometric mean,
and on the dense 1M-point scan, where the default grid is already the best
measured one, its choice must not be slower than the default beyond 1 %.
"""
import math
import os

import numpy as np
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

MODEL = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2606_06255_amd",
                     "param_mlp.npz")

# fresh clouds: (index, points); even index room-like, odd LiDAR-like
FRESH = [(0, 11000), (1, 18000), (2, 30000), (3, 52000), (4, 90000), (5, 150000), (6, 260000), (7, 450000),
         (8, 24000), (9, 70000), (10, 200000), (11, 700000)]
FRESH_SEED = 777


def _time(rf, x, m, n_vox, shell, reps):
    idx = None
    out_i = torch.empty(m, dtype=torch.int32, device=x.device)
    out_d = torch.empty(m, dtype=torch.float32, device=x.device)
    ts = []
    for r in range(reps + 1):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        idx = rf.build_index(x, n_vox=n_vox, shell=shell, reuse=idx)
        rf.sample(idx, m, 0, out_idx=out_i, out_d2=out_d)
        b.record()
        torch.cuda.synchronize()
        if r:
            ts.append(a.elapsed_time(b))
    assert rf.read_status(idx) == 0
    return float(np.median(ts)), out_i.cpu().numpy()


@pytest.fixture(scope="module")
def model():
    if not os.path.exists(MODEL):
        raise RuntimeError("the package ships no trained model (param_mlp.npz)")
    from paper_2606_06255_amd import param_model
    return param_model.ParamModel(torch.device("cuda:0"))


def test_network_gain_on_fresh_clouds(model, oracle_lib):
    import paper_2606_06255_amd as rf
    from paper_2606_06255_amd import param_model
    dev = torch.device("cuda:0")
    logs = []
    for i, n in FRESH:
        P = param_model.make_cloud(FRESH_SEED, i, n)
        m = n // 4
        x = torch.from_numpy(P).to(dev)
        nv, sh, k, _ = model.choose(x)
        nv0 = rf.default_n_vox(n)
        t0, i0 = _time(rf, x, m, nv0, 0.0, reps=5)
        t1, i1 = _time(rf, x, m, nv, sh, reps=5)
        assert np.array_equal(i0, i1), "the network's grid changed the sequence"
        ref, _ = oracle_lib.fps(P, min(m, 2000), 0, threads=0)
        assert np.array_equal(i1[:ref.size], ref)
        logs.append(math.log(t0 / t1))
        print("cloud %d N=%d: default n_vox %d %.2f ms; network (n_vox %d, shell %g) %.2f ms; %.3fx" % (
            i, n, nv0, t0, nv, sh, t1, t0 / t1))
    gain = math.exp(float(np.mean(logs)))
    print("geometric-mean gain over the default rule on %d fresh clouds: %.3fx" % (len(FRESH), gain))
    assert gain >= 1.05


def test_network_holds_the_default_on_dense_scan(model):
    import paper_2606_06255_amd as rf
    dev = torch.device("cuda:0")
    P = synth.dense_lidar(0)
    n, m = P.shape[0], 65536
    x = torch.from_numpy(P).to(dev)
    nv, sh, k, _ = model.choose(x)
    nv0 = rf.default_n_vox(n)
    if (nv, sh) == (nv0, 0.0):
        print("dense scan: the network keeps the default grid (n_vox %d)" % nv0)
        return
    # alternate the two grids so that drifts of the clock hit both alike
    t0s, t1s = [], []
    for _ in range(3):
        t0, i0 = _time(rf, x, m, nv0, 0.0, reps=3)
        t1, i1 = _time(rf, x, m, nv, sh, reps=3)
        t0s.append(t0)
        t1s.append(t1)
    assert np.array_equal(i0, i1)
    t0, t1 = float(np.median(t0s)), float(np.median(t1s))
    print("dense scan: default n_vox %d %.3f ms; network (n_vox %d, shell %g) %.3f ms" % (nv0, t0, nv, sh, t1))
    assert t1 <= 1.01 * t0
