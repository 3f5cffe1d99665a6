"""Pins of the FP64 reference of the voxel-parameter network (oracle/mlp_ref.py):
finite differences, closed forms and brute force, none of which reuse the
reference's own formulas."""
import os

import numpy as np
import pytest

from oracle import mlp_ref as R


def _nearest_bf16(x):
    """bfloat16 rounding by search: the two bf16 neighbours of x, then the
    nearer one, ties to the even mantissa."""
    out = []
    for v in np.asarray(x, dtype=np.float32).ravel():
        u = int(np.float32(v).view(np.uint32))
        lo = u & 0xFFFF0000
        hi = lo + 0x10000
        flo = np.uint32(lo).view(np.float32).astype(np.float64)
        fhi = np.uint32(hi).view(np.float32).astype(np.float64)
        d_lo, d_hi = abs(float(v) - flo), abs(fhi - float(v))
        if d_lo < d_hi or (d_lo == d_hi and ((lo >> 16) & 1) == 0):
            out.append(flo)
        else:
            out.append(fhi)
    return np.array(out)


def test_bf16_closed_forms():
    one = 1.0
    assert R.bf16_round(one) == 1.0
    assert R.bf16_round(1.0 + 2.0 ** -8) == 1.0                       # tie, even neighbour below
    assert R.bf16_round(1.0 + 3 * 2.0 ** -8) == 1.0 + 2 * 2.0 ** -7   # tie, even neighbour above
    assert R.bf16_round(1.0 + 2.0 ** -8 + 2.0 ** -20) == 1.0 + 2.0 ** -7
    assert R.bf16_round(-3.0) == -3.0
    assert R.bf16_round(0.0) == 0.0


def test_bf16_matches_search():
    rng = np.random.default_rng(0)
    x = np.concatenate([rng.standard_normal(3000).astype(np.float32) * 10.0 ** rng.integers(-6, 6, 3000),
                        rng.standard_normal(500).astype(np.float32)])
    assert np.array_equal(R.bf16_round(x).ravel(), _nearest_bf16(x))


def test_features_brute_force():
    # eight points at the corners of [0, 8]^3 and one in the middle
    pts = np.array([[x, y, z] for z in (0, 8) for y in (0, 8) for x in (0, 8)] + [[4, 4, 4]], dtype=np.float32)
    f, counts = R.features(pts)
    assert counts.sum() == 9
    # the edge is 8 * (1 + 1e-4) / 8 > 1: coordinate 8 lands in cell 7, 4 in cell 3
    for (x, y, z) in pts:
        cx, cy, cz = [min(7, int(v // (1.0001))) for v in (x, y, z)]
        assert counts[(cz * 8 + cy) * 8 + cx] >= 1
    assert counts[0] == 1 and counts[511] == 1 and counts[(3 * 8 + 3) * 8 + 3] == 1
    assert f[0] == np.float32((np.log(9.0) - 11.0) / 2.0)
    assert np.allclose(f[1:4], np.log1p(8.0) / 2.0)
    assert np.isclose(np.expm1(f[4:].astype(np.float64)).sum(), 64.0)
    assert f[4] == np.float32(np.log1p(64.0 / 9.0))


def test_features_uniform_cube():
    rng = np.random.default_rng(1)
    pts = rng.random((512 * 400, 3), dtype=np.float32)
    f, counts = R.features(pts)
    assert counts.sum() == pts.shape[0]
    assert counts.min() > 300 and counts.max() < 500
    assert abs(np.expm1(f[4:].astype(np.float64)).mean() - 0.125) < 1e-6


def test_features_degenerate_cloud():
    f, counts = R.features(np.ones((10, 3), dtype=np.float32))
    assert counts[0] == 10 and counts.sum() == 10
    assert np.all(f[1:4] == 0.0)


def _problem(seed, B=6):
    rng = np.random.default_rng(seed)
    theta = rng.standard_normal(R.N_PARAMS) * 0.1
    X = rng.standard_normal((B, R.F_IN)).astype(np.float32)
    T = rng.standard_normal((B, R.OUT))
    Wt = rng.random((B, R.OUT))
    return theta, X, T, Wt


def test_gradient_finite_differences():
    theta, X, T, Wt = _problem(2)
    g, L = R.gradient(theta, X, T, Wt, quantize=False)
    assert np.isclose(L, R.loss(theta, X, T, Wt, quantize=False))
    rng = np.random.default_rng(3)
    # a few coordinates of every parameter block
    o = 0
    picks = []
    for name, shape in R.SHAPES:
        size = int(np.prod(shape))
        picks += list(o + rng.choice(size, 6, replace=False))
        o += size
    h = 1e-6
    for k in picks:
        e = np.zeros_like(theta)
        e[k] = h
        fd = (R.loss(theta + e, X, T, Wt, False) - R.loss(theta - e, X, T, Wt, False)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(g[k])), (k, fd, g[k])


def test_gradient_passes_rounding_straight_through():
    theta, X, T, Wt = _problem(4)
    P = R.unpack(theta.copy())
    q = theta.copy()
    Q = R.unpack(q)
    for k in ("W1", "W2", "W3"):
        Q[k][...] = R.bf16_round(P[k])
    for k in ("b1", "b2", "b3"):
        Q[k][...] = np.asarray(P[k], dtype=np.float32)
    g1, L1 = R.gradient(theta, X, T, Wt)
    g2, L2 = R.gradient(q, X, T, Wt, quantize=False)
    assert np.array_equal(g1, g2) and L1 == L2


def test_relu_kink_and_zero_weights():
    # with all weights zero the network outputs its last bias and only the
    # last layer's bias has a gradient
    theta = np.zeros(R.N_PARAMS)
    P = R.unpack(theta)
    P["b3"][...] = np.arange(R.OUT) / 100.0
    X = np.ones((3, R.F_IN), dtype=np.float32)
    T = np.zeros((3, R.OUT))
    Wt = np.ones((3, R.OUT))
    Y, _ = R.forward(theta, X)
    assert np.allclose(Y, np.arange(R.OUT)[None, :] / 100.0)
    g, _ = R.gradient(theta, X, T, Wt)
    G = R.unpack(g)
    assert np.allclose(G["b3"], 2.0 * np.arange(R.OUT) / 100.0)
    for k in ("W1", "b1", "W2", "b2", "W3"):
        assert not G[k].any()


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(5)
    theta = rng.standard_normal(50)
    g = rng.standard_normal(50)
    new, m, v = R.adam(theta, np.zeros(50), np.zeros(50), g, 1, 1e-3)
    # bias-corrected first step: m_hat = g, v_hat = g^2
    assert np.allclose(new, theta - 1e-3 * g / (np.abs(g) + 1e-8))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_candidates():
    assert R.N_CAND == 36 and R.OUT == 72 and R.N_PARAMS == 41928
    assert R.candidate(0) == (12, 0.0) and R.candidate(35) == (192, 20.0)
    assert len({R.candidate(k) for k in range(R.N_CAND)}) == 36


# ---------------------------------------------------------------------------
# The forward pass against a network worked out by hand
# (tests/golden/mlp_forward_tiny.txt): power-of-two weights, negative
# pre-activations at both hidden layers, every output exact in FP64.
# ---------------------------------------------------------------------------
GOLDEN_MLP = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "mlp_forward_tiny.txt")


def _golden_network():
    P = {name: np.zeros(shape) for name, shape in R.SHAPES}
    X = np.zeros((2, R.F_IN), dtype=np.float32)
    Y = None
    rows = []
    for line in open(GOLDEN_MLP):
        line = line.split("#")[0].split()
        if not line:
            continue
        tag, rest = line[0], line[1:]
        if tag in ("W1", "W2", "W3"):
            P[tag][int(rest[0]), int(rest[1])] = float(rest[2])
        elif tag in ("b1", "b2", "b3"):
            P[tag][int(rest[0])] = float(rest[1])
        elif tag == "X":
            X[int(rest[0]), int(rest[1])] = float(rest[2])
        elif tag == "Y":
            rows.append((int(rest[0]), int(rest[1]), float(rest[2])))
    Y = np.tile(P["b3"], (2, 1))
    for b, k, v in rows:
        Y[b, k] = v
    theta = np.concatenate([P[name].ravel() for name, _ in R.SHAPES])
    return theta, X, Y, P


def test_forward_matches_hand_derived_network():
    theta, X, Y, _ = _golden_network()
    for quantize in (True, False):
        out, _ = R.forward(theta, X, quantize=quantize)
        assert np.array_equal(out, Y)


def test_hand_derived_network_separates_relu_mistakes():
    """The fixture is sharp enough: a forward pass without either hidden
    ReLU, or with one on the output, disagrees with it."""
    theta, X, Y, P = _golden_network()
    Xd = X.astype(np.float64)

    def fwd(relu1, relu2, relu_out):
        act = lambda z, on: np.maximum(z, 0.0) if on else z  # noqa: E731
        a1 = act(Xd @ P["W1"].T + P["b1"], relu1)
        a2 = act(a1 @ P["W2"].T + P["b2"], relu2)
        return act(a2 @ P["W3"].T + P["b3"], relu_out)

    assert np.array_equal(fwd(True, True, False), Y)
    for variant in ((False, True, False), (True, False, False), (True, True, True)):
        assert not np.array_equal(fwd(*variant), Y)
