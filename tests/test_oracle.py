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


# ---------------------------------------------------------------------------
# Euclidean mode: FPS over the FP32 norm (the rounded root of the squared
# distance), the distance of the update rule of Sec. 3.4.3.
# ---------------------------------------------------------------------------

def test_sqrt_rn_exact_is_round_to_nearest(oracle_lib):
    # Definition of rounding to nearest: r is the FP32 value whose neighbour
    # midpoints bracket sqrt(v), i.e. lo^2 < v < hi^2, checked in exact
    # rational arithmetic.  Covers subnormal inputs, powers of two (where the
    # lower neighbour is closer) and the top of the range.
    from fractions import Fraction
    rng = np.random.default_rng(7)
    vals = [np.float32(1.4e-45), np.float32(1.1754942e-38), np.float32(1.17549435e-38), np.float32(1.0),
            np.float32(2.0), np.float32(4.0), np.float32(0.25), np.finfo(np.float32).max]
    vals += list(rng.random(300, dtype=np.float32) * np.float32(4.0))
    vals += list(np.float32(2.0) ** rng.integers(-140, 127, 300).astype(np.float32)
                 * rng.random(300, dtype=np.float32).astype(np.float32) + np.float32(1e-45))
    for v in vals:
        v = np.float32(v)
        r = oracle_lib.sqrt_rn_exact(v)
        up = np.nextafter(r, np.float32(np.inf))
        dn = np.nextafter(r, np.float32(0))
        lo = (Fraction(float(dn)) + Fraction(float(r))) / 2
        hi = (Fraction(float(r)) + Fraction(float(up))) / 2
        assert lo * lo < Fraction(float(v)) < hi * hi, v
    assert oracle_lib.sqrt_rn_exact(np.float32(0)) == 0
    assert np.isinf(oracle_lib.sqrt_rn_exact(np.float32(np.inf)))


def test_euclid_lattice_closed_form(oracle_lib):
    # On the integer lattice 0..16 every squared distance is a perfect
    # square, so the Euclidean order has no rounding and the picks are those
    # of the squared form; the distances are the integer gaps.
    x = np.arange(17, dtype=np.float32)
    P = np.stack([x, 0 * x, 0 * x], 1)
    idx, d = oracle_lib.fps(P, 17, 0, euclid=True)
    assert idx.tolist() == [0, 16, 8, 4, 12, 2, 6, 10, 14, 1, 3, 5, 7, 9, 11, 13, 15]
    assert d.tolist() == [np.inf, 16, 8, 4, 4, 2, 2, 2, 2, 1, 1, 1, 1, 1, 1, 1, 1]


def _rounding_tie_pair(seed):
    """Two points at different FP32 squared distances from the origin whose
    rounded roots are equal.  For p1 = (u, v, 0) with d2 = A and r the
    rounded root of A, the axis point p2 = (r, 0, 0) has d2 = fl(r^2), whose
    rounded root is r again (radix 2, round to nearest); it differs from A
    for most u, v."""
    import oracle
    rng = np.random.default_rng(seed)
    while True:
        u, v = rng.random(2, dtype=np.float32) + np.float32(0.5)
        A = (u * u) + (v * v)
        r = oracle.sqrt_rn_exact(A)
        B = r * r
        if A != B and oracle.sqrt_rn_exact(B) == r:
            return (u, v), r, A, B


@pytest.mark.parametrize("seed", range(6))
def test_euclid_rounding_tie_takes_lower_index(oracle_lib, seed):
    (u, v), r, A, B = _rounding_tie_pair(seed)
    lo_pt, hi_pt = ((u, v, 0), (r, 0, 0)) if A < B else ((r, 0, 0), (u, v, 0))
    # index 1 holds the smaller squared distance, index 2 the larger
    P = np.array([(0, 0, 0), lo_pt, hi_pt], dtype=np.float32)
    idx_sq, d_sq = oracle_lib.fps(P, 2, 0)
    idx_eu, d_eu = oracle_lib.fps(P, 2, 0, euclid=True)
    assert idx_sq.tolist() == [0, 2] and d_sq[1] == max(A, B)
    assert idx_eu.tolist() == [0, 1] and d_eu[1] == r
    assert same((idx_eu, d_eu), oracle_lib.fps_bruteforce(P, 2, 0, euclid=True))


def test_euclid_bruteforce_tiny(oracle_lib):
    rng = np.random.default_rng(4321)
    diverged = 0
    for t in range(240):
        n = int(rng.integers(1, 41))
        kind = t % 3
        if kind == 0:
            P = rng.random((n, 3), dtype=np.float32)
        elif kind == 1:   # grid of step 0.1: equal real distances, unequal FP32 ones
            P = rng.integers(-4, 5, size=(n, 3)).astype(np.float32) * np.float32(0.1)
        else:             # wide dynamic range
            P = (rng.normal(size=(n, 3)) * 10.0 ** rng.integers(-3, 4)).astype(np.float32)
        m = int(rng.integers(1, n + 1))
        s = int(rng.integers(0, n))
        ref = oracle_lib.fps(P, m, s, euclid=True)
        assert same(ref, oracle_lib.fps_bruteforce(P, m, s, euclid=True)), (t, n, m, s)
        assert same(ref, oracle_lib.fps_numpy(P, m, s, euclid=True)), (t, n, m, s)
        diverged += not np.array_equal(ref[0], oracle_lib.fps(P, m, s)[0])
    assert diverged >= 10   # the cases really exercise rounding ties


def test_euclid_against_squared_first_divergence(oracle_lib):
    # The rounded root is non-decreasing, so the two orders agree up to the
    # first pick where two squared distances share one rounded root; there
    # the Euclidean form takes the lower index of the tied points, and until
    # then its distances are the rounded roots of the squared ones.
    rng = np.random.default_rng(11)
    seen = 0
    for t in range(8):
        P = rng.integers(-40, 41, size=(3000, 3)).astype(np.float32) * np.float32(0.1)
        m = 800
        i_sq, d_sq = oracle_lib.fps(P, m, 0, threads=0)
        i_eu, d_eu = oracle_lib.fps(P, m, 0, threads=0, euclid=True)
        k = int(np.argmax(i_sq != i_eu)) if np.any(i_sq != i_eu) else m
        assert np.array_equal(d_eu[1:k], oracle_lib._roots_exact(d_sq[1:k]))
        if k < m:
            seen += 1
            # after k-1 equal picks both states are equal up to the root
            S = P[i_sq[:k]]
            dd = P[:, None, :] - S[None, :, :]
            sq = dd * dd
            D = ((sq[..., 0] + sq[..., 1]) + sq[..., 2]).min(axis=1)
            R = oracle_lib._roots_exact(D)
            top = R.max()
            tied = np.flatnonzero(R == top)
            assert i_eu[k] == tied[0] and d_eu[k] == top
            assert D[i_sq[k]] == D.max() and i_sq[k] != tied[0]
    assert seen >= 1


def test_euclid_invariants_room(oracle_lib):
    P = synth.room(3)[:12000]
    m = 1500
    idx, d = oracle_lib.fps(P, m, 0, threads=0, euclid=True)
    assert idx[0] == 0 and np.isinf(d[0])
    assert np.all(d[1:-1] >= d[2:])
    assert len(set(idx.tolist())) == m
    S = P[idx[:-1]]
    near = np.full(P.shape[0], np.inf, np.float32)
    for s in S:
        dd = P - s
        sq = dd * dd
        near = np.minimum(near, np.sqrt((sq[:, 0] + sq[:, 1]) + sq[:, 2]))
    assert near.max() == d[-1]
