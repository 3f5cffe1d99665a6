"""Pins of the plain FPS oracle against facts that do not come from the oracle itself.

- a hand-derived closed form (tests/golden/lattice_1d_17.txt) and its
  generalisation to the lattice 0..2^k;
- the selection rule of Sec. 3.1 evaluated from scratch on tiny clouds;
- the paper's Euclidean definition in exact integer arithmetic on integer clouds;
- invariants of Algorithm 1 (non-increasing distances, covering, distinct picks);
- exact symmetries of the FP32 formula (x<->y swap, axis negation, scaling by 2^k);
- prefix nesting of multi-stage FPS;
- degenerate inputs and argument errors.
"""
import os

import numpy as np
import pytest

import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def bits(a):
    return np.asarray(a, dtype=np.float32).view(np.uint32)


def same(a, b):
    return np.array_equal(a[0], b[0]) and np.array_equal(bits(a[1]), bits(b[1]))


def read_golden(name):
    out = {}
    for line in open(os.path.join(GOLD, name)):
        if line.startswith("#") or not line.strip():
            continue
        k, *v = line.split()
        out[k] = v
    return out


def test_lattice_golden(oracle_lib):
    g = read_golden("lattice_1d_17.txt")
    x = np.arange(17, dtype=np.float32)
    P = np.stack([x, 0 * x, 0 * x], 1)
    idx, d2 = oracle_lib.fps(P, 17, 0)
    assert idx.tolist() == [int(v) for v in g["idx"]]
    assert d2.tolist() == [float(v) for v in g["d2"]]


@pytest.mark.parametrize("k", [1, 2, 3, 5, 7])
def test_lattice_closed_form(oracle_lib, k):
    # On 0..2^k (start 0): 2^k first, then for level l = 1..k the odd multiples
    # of 2^(k-l) in increasing order, each at squared distance 4^(k-l).
    n = 2 ** k + 1
    exp_idx, exp_d2 = [0, 2 ** k], [np.inf, 4.0 ** k]
    for lev in range(1, k + 1):
        step = 2 ** (k - lev)
        for q in range(step, 2 ** k, 2 * step):
            exp_idx.append(q)
            exp_d2.append(float(step * step))
    x = np.arange(n, dtype=np.float32)
    for axis in range(3):
        P = np.zeros((n, 3), np.float32)
        P[:, axis] = x
        idx, d2 = oracle_lib.fps(P, n, 0)
        assert idx.tolist() == exp_idx
        assert d2.tolist() == exp_d2


def test_bruteforce_tiny(oracle_lib):
    rng = np.random.default_rng(1234)
    for t in range(1500):
        n = int(rng.integers(1, 49))
        kind = t % 4
        if kind == 0:
            P = rng.random((n, 3), dtype=np.float32)
        elif kind == 1:   # coarse values -> many exact ties and duplicates
            P = rng.integers(0, 4, size=(n, 3)).astype(np.float32)
        elif kind == 2:   # clustered, wide dynamic range
            P = (rng.normal(size=(n, 3)) * 10.0 ** rng.integers(-3, 4)).astype(np.float32)
        else:             # planar
            P = rng.random((n, 3), dtype=np.float32)
            P[:, 2] = 0.5
        m = int(rng.integers(1, n + 1))
        s = int(rng.integers(0, n))
        assert same(oracle_lib.fps(P, m, s), oracle_lib.fps_bruteforce(P, m, s)), (t, n, m, s)


def test_exact_integer_definition(oracle_lib):
    rng = np.random.default_rng(99)
    for t in range(60):
        n = int(rng.integers(2, 200))
        hi = int(rng.choice([3, 8, 64, 1000]))
        P = rng.integers(-hi, hi, size=(n, 3))
        if t % 5 == 0:
            P[:, 1:] = 0
        m = int(rng.integers(1, n + 1))
        s = int(rng.integers(0, n))
        idx, d2 = oracle_lib.fps(P.astype(np.float32), m, s)
        eidx, ed2 = oracle_lib.fps_exact_int(P.tolist(), m, s)
        assert idx.tolist() == eidx
        assert np.isinf(d2[0]) and d2[1:].astype(np.int64).tolist() == ed2[1:]


def test_numpy_transcription_and_threads(oracle_lib):
    a = synth.cube(5)
    r = synth.room(2)[:20000]
    for P, m in ((a, 1024), (r, 600)):
        ref = oracle_lib.fps(P, m, 0, threads=1)
        assert same(ref, oracle_lib.fps_numpy(P, m, 0))
        assert same(ref, oracle_lib.fps(P, m, 0, threads=4))
        assert same(ref, oracle_lib.fps(P, m, 0, threads=0))


def invariants(P, m, start, idx, d2):
    assert idx[0] == start and np.isinf(d2[0])
    assert np.all(d2[1:-1] >= d2[2:])                       # non-increasing
    pos = d2 > 0
    assert len(set(idx[pos].tolist())) == int(pos.sum())    # distinct while d2 > 0
    # covering: every point is within the last reported distance of the first m-1 picks
    S = P[idx[:-1]]
    near = np.full(P.shape[0], np.inf, np.float32)
    for s in S:
        d = P - s
        sq = d * d
        near = np.minimum(near, (sq[:, 0] + sq[:, 1]) + sq[:, 2])
    assert near.max() <= d2[-1]
    assert near.max() == d2[-1] or m == 1


def test_invariants_room_lidar(oracle_lib):
    for P, m in ((synth.room(1)[:12000], 800), (synth.lidar(1)[::8], 700), (synth.cube(1), 1024)):
        idx, d2 = oracle_lib.fps(P, m, 0)
        invariants(P, m, 0, idx, d2)


def test_symmetries(oracle_lib):
    P = synth.room(3)[:6000]
    m = 500
    idx, d2 = oracle_lib.fps(P, m, 7)
    Q = P[:, [1, 0, 2]].copy()                       # x <-> y (addition commutes)
    assert same((idx, d2), oracle_lib.fps(Q, m, 7))
    for a in range(3):                               # negating an axis
        Q = P.copy()
        Q[:, a] = -Q[:, a]
        assert same((idx, d2), oracle_lib.fps(Q, m, 7))
    for k in (-3, 2, 5):                             # scaling by 2^k scales d2 by 4^k exactly
        i2, e2 = oracle_lib.fps(P * np.float32(2.0 ** k), m, 7)
        assert np.array_equal(i2, idx)
        assert np.array_equal(e2[1:], d2[1:] * np.float32(4.0 ** k))


def test_prefix_nesting_multistage(oracle_lib):
    P = synth.lidar(2)[::4]
    sizes = [P.shape[0] // 4, P.shape[0] // 16, P.shape[0] // 64]
    idx1, d1 = oracle_lib.fps(P, sizes[0], 0)
    cur = P[idx1]
    for m in sizes[1:]:
        i2, e2 = oracle_lib.fps(cur, m, 0)
        assert np.array_equal(i2, np.arange(m))
        assert np.array_equal(bits(e2), bits(d1[:m]))
        cur = cur[i2]


def test_degenerate(oracle_lib):
    P = np.ones((50, 3), np.float32)
    idx, d2 = oracle_lib.fps(P, 10, 3)
    assert idx.tolist() == [3] + [0] * 9 and d2[1:].tolist() == [0.0] * 9
    idx, d2 = oracle_lib.fps(np.zeros((1, 3), np.float32), 1, 0)
    assert idx.tolist() == [0]
    # duplicates: a duplicate of a chosen point is never picked while others are farther
    P = np.array([[0, 0, 0], [1, 0, 0], [0, 0, 0], [1, 0, 0], [5, 0, 0]], np.float32)
    idx, d2 = oracle_lib.fps(P, 5, 0)
    assert idx.tolist() == [0, 4, 1, 0, 0] and d2.tolist() == [np.inf, 25, 1, 0, 0]


def test_argument_errors(oracle_lib):
    P = synth.cube(0)[:10]
    for m, s in ((11, 0), (0, 0), (3, 10), (3, -1)):
        with pytest.raises(oracle_lib.OracleError):
            oracle_lib.fps(P, m, s)
    Q = P.copy()
    Q[4, 1] = np.nan
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.fps(Q, 3, 0)
    Q[4, 1] = np.inf
    with pytest.raises(oracle_lib.OracleError):
        oracle_lib.fps(Q, 3, 0)
