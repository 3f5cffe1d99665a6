"""The pruning bound the samplers use (prune_bound.h), on the CPU.

Sec. 3.4.2 proves in real arithmetic that a voxel whose sphere lies at least
sqrt(Dist_v) beyond its radius from the new sample cannot change.  The
library skips a tile when fl32(||s - c||^2) >= thr(R, Dist_v).  These tests
check that decision against an exact rational evaluation of the bound with
the FP32 rounding of the distance formula made explicit, at placements
within a few ulps of the boundary, and that a members-on-the-sphere witness
never shows a skipped tile whose point would have been updated.  The same
formula with its margins removed (a planted mistake) must be caught.
"""
import ctypes
import os
import subprocess
from fractions import Fraction

import numpy as np
import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
U = Fraction(1, 2 ** 24)          # unit roundoff of FP32
LOSS5 = (1 - U) ** 5              # FP32 squared distance >= LOSS5 * exact


@pytest.fixture(scope="module")
def shim(tmp_path_factory):
    out = str(tmp_path_factory.mktemp("prune") / "libprune_shim.so")
    subprocess.run(["g++", "-O2", "-std=c++17", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                    "-Wall", "-o", out, os.path.join(HERE, "native", "prune_shim.cpp")], check=True)
    L = ctypes.CDLL(out)
    f = ctypes.c_float
    L.shim_prune_threshold.argtypes = [f, f]
    L.shim_prune_threshold.restype = f
    L.shim_prune_threshold_with.argtypes = [f, f, f, f]
    L.shim_prune_threshold_with.restype = f
    return L


def f32(v):
    return np.float32(v)


def sqdist32(p, s):
    """((dx*dx + dy*dy) + dz*dz) in FP32, one rounding per operation."""
    d = [f32(f32(p[a]) - f32(s[a])) for a in range(3)]
    sq = [f32(x * x) for x in d]
    return f32(f32(sq[0] + sq[1]) + sq[2])


def exact_safe(s, c, R, dv):
    """True when every point within exact distance R of c has an FP32
    squared distance to s of at least dv: ||s - c|| - R >= sqrt(dv / LOSS5),
    decided in rational arithmetic (no rounding anywhere)."""
    dv = Fraction(float(dv))
    if dv == 0:
        return True
    D2 = sum((Fraction(float(s[a])) - Fraction(float(c[a]))) ** 2 for a in range(3))
    R = Fraction(float(R))
    K = dv / LOSS5
    if D2 < R * R:
        return False
    A = D2 + R * R - K
    return A >= 0 and A * A >= 4 * R * R * D2


def sphere_member(s, c, R):
    """An FP32 point within exact distance R of c, on the segment towards s
    as far as FP32 allows: the member of a tile closest to the sample."""
    c64 = np.array([float(v) for v in c])
    dirn = np.array([float(v) for v in s]) - c64
    nrm = np.linalg.norm(dirn)
    if nrm == 0:
        return [f32(v) for v in c]
    for shrink in range(64):
        t = float(R) * (1.0 - shrink * 2.0 ** -23)
        p = [f32(c64[a] + dirn[a] / nrm * t) for a in range(3)]
        e2 = sum((Fraction(float(p[a])) - Fraction(float(c[a]))) ** 2 for a in range(3))
        if e2 <= Fraction(float(R)) ** 2:
            return p
    return [f32(v) for v in c]


def near_members(s, c, R, count=8, seed=1):
    """The member closest to s and members on the sphere in directions
    jittered by about 2^-13 around it (FP32 rounding of the sample then
    falls differently)."""
    out = [sphere_member(s, c, R)]
    c64 = np.array([float(v) for v in c])
    dirn = np.array([float(v) for v in s]) - c64
    nrm = np.linalg.norm(dirn)
    if nrm == 0:
        return out
    rng = np.random.default_rng(seed)
    for _ in range(count):
        dd = dirn / nrm + rng.standard_normal(3) * 2.0 ** -13
        dd /= np.linalg.norm(dd)
        out.append(sphere_member([f32(c64[a] + dd[a] * nrm) for a in range(3)], c, R))
    return out


def cases(seed=0):
    """Tile sphere (c, R), tile distance dv and a sample s placed at
    R + sqrt(dv) times (1 + k 2^-24), k in [-48, 48], across scales from
    2^-50 to 2^50 and at the ends of the accepted range of dv."""
    rng = np.random.default_rng(seed)
    out = []
    for sigma in (2.0 ** -50, 2.0 ** -10, 1.0, 37.0, 2.0 ** 40, 2.0 ** 50):
        for dv_rel in (1.0, 0.37, 2.9):
            dv = f32(sigma * sigma * dv_rel)
            if not (2.0 ** -100 <= float(dv) <= 2.0 ** 100):
                continue
            for R_rel in (0.0, 0.25, 1.0, 3.0):
                R = f32(sigma * R_rel)
                for _ in range(6):
                    c = [f32(v) for v in sigma * rng.uniform(-2, 2, 3)]
                    d = rng.standard_normal(3)
                    d /= np.linalg.norm(d)
                    tstar = float(R) + float(np.sqrt(np.float64(dv)))
                    for k in range(-48, 49, 3):
                        t = tstar * (1.0 + k * 2.0 ** -24)
                        s = [f32(float(c[a]) + d[a] * t) for a in range(3)]
                        out.append((s, c, R, dv, k))
    # the ends of the range of dv: 2^-100 and 2^100 are accepted, values
    # beyond them give NaN (never skip)
    for dv, sigma in ((f32(2.0 ** -100), 2.0 ** -50), (f32(2.0 ** 100), 2.0 ** 50)):
        for R_rel in (0.0, 1.0):
            R = f32(sigma * R_rel)
            c = [f32(0.0)] * 3
            tstar = float(R) + float(np.sqrt(np.float64(dv)))
            for k in range(-48, 49):
                t = tstar * (1.0 + k * 2.0 ** -24)
                out.append(([f32(t), f32(0.0), f32(0.0)], c, R, dv, k))
    return out


def violations(thr_fn, cs):
    """(skips, exact-bound violations, member witnesses): a witness is a
    skipped tile whose on-sphere member would still be updated."""
    skips = bad_exact = bad_member = 0
    for s, c, R, dv, _ in cs:
        thr = f32(thr_fn(float(R), float(dv)))
        q = sqdist32(c, s)
        if not (q >= thr):
            continue
        skips += 1
        if not exact_safe(s, c, R, dv):
            bad_exact += 1
        if any(sqdist32(p, s) < dv for p in near_members(s, c, R)):
            bad_member += 1
    return skips, bad_exact, bad_member


def test_special_values(shim):
    T = shim.shim_prune_threshold
    assert T(1.0, 0.0) == 0.0                      # nothing can decrease: always skip
    assert T(0.0, 0.0) == 0.0
    for dv in (2.0 ** -101, np.float32(2.0 ** -100) * np.float32(1 - 2.0 ** -24), 2.0 ** 101,
               float(np.float32(2.0 ** 100) * np.float32(1 + 2.0 ** -23)), float("inf"), float("nan")):
        assert np.isnan(T(1.0, dv))                # outside [2^-100, 2^100]: never skip
    assert np.isfinite(T(0.0, 2.0 ** -100)) and np.isfinite(T(2.0 ** 50, 2.0 ** 100))
    assert np.isnan(T(2e19, 1.0))                  # the square would overflow: never skip


def test_threshold_dominates_the_exact_bound(shim):
    """thr >= (R + sqrt(dv / (1 - 2^-20)))^2 (1 + 2^-20), checked exactly."""
    rng = np.random.default_rng(5)
    for _ in range(3000):
        e = rng.integers(-45, 45)
        dv = f32(rng.uniform(0.5, 2.0) * 2.0 ** (2 * e))
        R = f32(rng.choice([0.0, rng.uniform(0, 4)]) * 2.0 ** e)
        thr = shim.shim_prune_threshold(float(R), float(dv))
        assert np.isfinite(thr)
        # thr >= (R + sqrt(K))^2 (1 + 2^-20), K = dv / (1 - 2^-20):  with
        # y = thr / (1 + 2^-20) - R^2 - K, need y >= 0 and y^2 >= 4 R^2 K
        K = Fraction(float(dv)) / (1 - Fraction(1, 2 ** 20))
        y = Fraction(float(thr)) / (1 + Fraction(1, 2 ** 20)) - Fraction(float(R)) ** 2 - K
        assert y >= 0 and y * y >= 4 * Fraction(float(R)) ** 2 * K


def test_skip_decisions_are_exactly_safe(shim):
    cs = cases()
    skips, bad_exact, bad_member = violations(shim.shim_prune_threshold, cs)
    assert bad_exact == 0 and bad_member == 0
    assert skips > len(cs) // 4                    # the bound does prune near the boundary
    # and it is tight: 64 ulps beyond the real-arithmetic boundary it always skips
    for s, c, R, dv, k in cs:
        if k >= 45:
            thr = f32(shim.shim_prune_threshold(float(R), float(dv)))
            assert sqdist32(c, s) >= thr


def test_zero_margin_variant_is_caught(shim):
    """The same formula without its margins (the bound of the paper's
    real-arithmetic proof, rounded up) skips tiles whose members would
    still be updated: the checks above must reject it."""
    cs = cases()
    zero = lambda R, dv: shim.shim_prune_threshold_with(R, dv, 1.0, 1.0)  # noqa: E731
    skips, bad_exact, bad_member = violations(zero, cs)
    assert bad_exact > 0
    assert bad_member > 0
