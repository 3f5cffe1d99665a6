"""The voxel-parameter network's HIP kernels (features, forward, gradient,
Adam step, choice) against the FP64 reference in oracle/mlp_ref.py, on
seeded inputs."""
import numpy as np
import pytest
import torch

import synth
from oracle import mlp_ref as R

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rf():
    import paper_2606_06255_amd as rf
    if not torch.cuda.is_available():
        raise RuntimeError("GPU tests need a GPU")
    return rf


@pytest.fixture(scope="module")
def dev():
    return torch.device("cuda:0")


def _theta(seed, scale=1.0):
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in R.SHAPES:
        fan_in = shape[1] if len(shape) == 2 else 64
        parts.append(rng.uniform(-1, 1, size=int(np.prod(shape))) * scale * np.sqrt(6.0 / fan_in))
    return np.concatenate(parts).astype(np.float32)


def _batch(seed, B):
    rng = np.random.default_rng(seed)
    X = np.concatenate([rng.normal(0, 1, (B, 4)), rng.exponential(0.125, (B, 512))], axis=1).astype(np.float32)
    T = rng.normal(0, 1, (B, R.OUT)).astype(np.float32)
    Wt = rng.random((B, R.OUT)).astype(np.float32)
    return X, T, Wt


@pytest.mark.parametrize("cloud", ["cube", "room", "lidar", "ones", "line"])
def test_features(rf, dev, cloud):
    pts = {"cube": lambda: synth.cube(0, 5000), "room": lambda: synth.room(1),
           "lidar": lambda: synth.lidar(2), "ones": lambda: np.ones((77, 3), dtype=np.float32),
           "line": lambda: np.stack([np.arange(300), np.zeros(300), np.zeros(300)], 1).astype(np.float32)}[cloud]()
    net = rf.MLP(dev)
    f = net.features(torch.from_numpy(pts).to(dev)).cpu().numpy()
    ref, counts = R.features(pts)
    # the cell counts are decided by FP64 bin comparisons on both sides: exact
    n = pts.shape[0]
    got_counts = np.rint(np.expm1(f[4:].astype(np.float64)) * n / 64.0).astype(np.int64)
    assert np.array_equal(got_counts, counts)
    assert np.allclose(f, ref, rtol=1e-6, atol=1e-7)


def test_features_nonfinite(rf, dev):
    pts = synth.cube(3, 1000)
    pts[17, 2] = np.inf
    net = rf.MLP(dev)
    f = net.features(torch.from_numpy(pts).to(dev)).cpu().numpy()
    assert np.isnan(f).all()


@pytest.mark.parametrize("B", [1, 7, 64, 333])
def test_forward(rf, dev, B):
    theta = _theta(B)
    X, _, _ = _batch(B + 1, B)
    net = rf.MLP(dev, rows=B)
    net.load(theta)
    y = net.forward(torch.from_numpy(X).to(dev)).cpu().numpy().astype(np.float64)
    ref, _ = R.forward(theta, X)
    scale = np.abs(ref).max()
    assert np.abs(y - ref).max() <= 1e-5 * scale


def test_save_roundtrip(rf, dev):
    theta = _theta(9)
    net = rf.MLP(dev)
    net.load(theta)
    assert np.array_equal(net.save(), theta)


@pytest.mark.parametrize("B,weighted", [(5, True), (128, False), (1000, True)])
def test_gradient(rf, dev, B, weighted):
    theta = _theta(20 + B)
    X, T, Wt = _batch(30 + B, B)
    if not weighted:
        Wt = np.ones_like(Wt)
    net = rf.MLP(dev, rows=B)
    net.load(theta)
    g, loss = net.gradient(torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev),
                           torch.from_numpy(Wt).to(dev) if weighted else None)
    g = g.cpu().numpy().astype(np.float64)
    gr, Lr = R.gradient(theta, X, T, Wt)
    assert abs(float(loss.item()) - Lr) <= 1e-5 * abs(Lr)
    o = 0
    for name, shape in R.SHAPES:
        size = int(np.prod(shape))
        a, b = g[o:o + size], gr[o:o + size]
        assert np.abs(a - b).max() <= 1e-3 * max(np.abs(b).max(), 1e-12), name
        assert np.linalg.norm(a - b) <= 1e-4 * np.linalg.norm(b), name
        o += size


def test_adam_steps_follow_reference(rf, dev):
    theta = _theta(41, 0.5)
    X, T, Wt = _batch(42, 96)
    Xd, Td, Wd = (torch.from_numpy(a).to(dev) for a in (X, T, Wt))
    net = rf.MLP(dev, rows=96)
    net.load(theta)
    ref = theta.astype(np.float64)
    m = np.zeros_like(ref)
    v = np.zeros_like(ref)
    lr = 1e-3
    for step in range(1, 4):
        g, _ = R.gradient(ref, X, T, Wt)
        ref, m, v = R.adam(ref, m, v, g, step, lr)
        net.train_step(Xd, Td, Wd, lr=lr)
        got = net.save().astype(np.float64)
        # Adam moves every parameter by about lr per step whatever the size of
        # its gradient, so a component within rounding of zero may move either
        # way on the two paths; all others must agree closely
        d = np.abs(got - ref)
        assert d.max() <= 2.5 * step * lr, step
        assert np.mean(d > 0.01 * lr) <= 1e-3, step
        assert d.mean() <= 1e-3 * lr, step


def test_training_reduces_loss(rf, dev):
    # a teacher network of the same shape provides learnable targets
    teacher = _theta(50)
    X, _, _ = _batch(51, 512)
    T, _ = R.forward(teacher, X)
    T = T.astype(np.float32)
    Xd, Td = torch.from_numpy(X).to(dev), torch.from_numpy(T).to(dev)
    net = rf.MLP(dev, rows=512)
    net.load(_theta(52))
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    net.train_step(Xd, Td, lr=2e-3, loss=loss)
    first = float(loss.item())
    for _ in range(300):
        net.train_step(Xd, Td, lr=2e-3, loss=loss)
    last = float(loss.item())
    assert last < 0.1 * first, (first, last)
    assert abs(R.loss(net.save(), X, T, np.ones_like(T)) - last) <= 0.05 * first


def test_choose(rf, dev):
    theta = _theta(60)
    net = rf.MLP(dev)
    net.load(theta)
    f = torch.from_numpy(_batch(61, 1)[0][0]).to(dev)
    y_ref, _ = R.forward(theta, f.cpu().numpy()[None, :])
    best = int(np.argmin(y_ref[0, :R.N_CAND]))
    for d in (0, 17, 35):
        c, y = net.choose(f, d, margin=0.0)
        assert c == best or (c == d and y_ref[0, d] <= y_ref[0, best] + 1e-5)
        c, _ = net.choose(f, d, margin=1e9)
        assert c == d
