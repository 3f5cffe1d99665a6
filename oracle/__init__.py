"""ORACLE -- test infrastructure, not product code.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It shares no code with the device path
(``paper_2606_06255_amd``) and never imports it.

Contents
--------
``fps``             plain FPS in C (Algorithm 1 of the paper, FP32 squared
                    distance, strict update, lowest-index tie-break);
                    ``euclid=True`` uses the FP32 Euclidean distance (the
                    rounded root of the squared one, Sec. 3.4.3).
``fps_numpy``       the same definition as a vectorised numpy loop (a second,
                    independent transcription used to cross-check the C code).
``fps_bruteforce``  the selection rule of Sec. 3.1 evaluated from scratch at
                    every step (min over the chosen set, then arg max), for
                    tiny clouds.
``fps_exact_int``   the paper's Euclidean definition on integer clouds with
                    exact integer arithmetic (no floating point at all).
``sqrt_rn_exact``   correctly rounded FP32 square root by integer arithmetic
                    (no library square root), for the Euclidean pins.
``rfps_cpu``        CPU RadiusFPS (Sec. 3) with telemetry; must equal ``fps``.
``voxelize``        the voxel grid of Sec. 3.2 (pmin, L, voxel id per point).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_SOURCES = ["fps_oracle.c", "cpu_rfps.c"]

# option bits of rfps_cpu_sample (cpu_rfps.c)
NO_PRUNE = 1
NO_SKIP = 2
PAPER_RADIUS = 4
MUT_CENTROID = 256
MUT_HALF_RADIUS = 512


class Telemetry(ctypes.Structure):
    _fields_ = [(k, ctypes.c_int64) for k in (
        "iters", "voxels", "voxel_tests", "voxels_pruned",
        "points_visited", "points_skipped", "points_updated")]

    def as_dict(self):
        return {k: int(getattr(self, k)) for k, _ in self._fields_}


def build(force: bool = True) -> str:
    """Compile liboracle.so with gcc (no fast-math, no FP contraction, OpenMP)."""
    srcs = [os.path.join(_HERE, s) for s in _SOURCES]
    if not force and os.path.exists(_LIB_PATH) and all(
            os.path.getmtime(_LIB_PATH) >= os.path.getmtime(s) for s in srcs):
        return _LIB_PATH
    tmp = _LIB_PATH + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-fPIC", "-shared", "-Wall", "-Wextra", "-o", tmp] + srcs + ["-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = ctypes.CDLL(_LIB_PATH)
        i64, i32, u32 = ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
        vp = ctypes.c_void_p
        L.oracle_fps.argtypes = [vp, i64, i64, i64, vp, vp, ctypes.c_int]
        L.oracle_fps.restype = ctypes.c_int
        L.oracle_fps_euclid.argtypes = [vp, i64, i64, i64, vp, vp, ctypes.c_int]
        L.oracle_fps_euclid.restype = ctypes.c_int
        L.oracle_num_threads.argtypes = []
        L.oracle_num_threads.restype = ctypes.c_int
        L.rfps_cpu_sample.argtypes = [vp, i64, i64, i64, i32, i32, u32, vp, vp,
                                      ctypes.POINTER(Telemetry)]
        L.rfps_cpu_sample.restype = ctypes.c_int
        L.rfps_cpu_voxelize.argtypes = [vp, i64, i32, vp, vp]
        L.rfps_cpu_voxelize.restype = ctypes.c_int
        _lib = L
    return _lib


class OracleError(RuntimeError):
    pass


def _as_xyz(xyz):
    a = np.ascontiguousarray(xyz, dtype=np.float32)
    if a.ndim != 2 or a.shape[1] != 3:
        raise ValueError("xyz must be [N,3]")
    return a


def fps(xyz, m: int, start: int = 0, threads: int = 1, euclid: bool = False):
    """Plain FPS oracle. Returns (idx int32 [m], d2 float32 [m]).

    With ``euclid`` the distances (state and output) are FP32 Euclidean
    norms instead of squared distances.
    """
    a = _as_xyz(xyz)
    idx = np.empty(m, dtype=np.int32)
    d2 = np.empty(m, dtype=np.float32)
    fn = lib().oracle_fps_euclid if euclid else lib().oracle_fps
    rc = fn(a.ctypes.data, a.shape[0], m, start, idx.ctypes.data, d2.ctypes.data, threads)
    if rc:
        raise OracleError("oracle_fps returned %d" % rc)
    return idx, d2


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def rfps_cpu(xyz, m: int, start: int = 0, n_vox: int = 16, tile: int = 0, opts: int = 0):
    """CPU RadiusFPS. Returns (idx, d2, telemetry dict)."""
    a = _as_xyz(xyz)
    idx = np.empty(m, dtype=np.int32)
    d2 = np.empty(m, dtype=np.float32)
    tel = Telemetry()
    rc = lib().rfps_cpu_sample(a.ctypes.data, a.shape[0], m, start, n_vox, tile, opts,
                               idx.ctypes.data, d2.ctypes.data, ctypes.byref(tel))
    if rc:
        raise OracleError("rfps_cpu_sample returned %d" % rc)
    return idx, d2, tel.as_dict()


def voxelize(xyz, n_vox: int):
    """Voxel grid of Sec. 3.2: returns (pmin float64[3], L, vid uint32[N])."""
    a = _as_xyz(xyz)
    g = np.empty(4, dtype=np.float64)
    vid = np.empty(a.shape[0], dtype=np.uint32)
    rc = lib().rfps_cpu_voxelize(a.ctypes.data, a.shape[0], n_vox, g.ctypes.data, vid.ctypes.data)
    if rc:
        raise OracleError("rfps_cpu_voxelize returned %d" % rc)
    return g[:3].copy(), float(g[3]), vid


# ---------------------------------------------------------------------------
# Pure-Python / numpy transcriptions (independent of the C code above).
# ---------------------------------------------------------------------------

def sqdist_np(P, s):
    """FP32 squared distance of every row of P to s: ((dx*dx + dy*dy) + dz*dz).

    numpy evaluates float32 element-wise arithmetic in IEEE single precision
    without contraction, one rounding per operation.
    """
    P = np.asarray(P, dtype=np.float32)
    s = np.asarray(s, dtype=np.float32)
    d = P - s[None, :]
    sq = d * d
    return (sq[:, 0] + sq[:, 1]) + sq[:, 2]


def fps_numpy(xyz, m: int, start: int = 0, euclid: bool = False):
    """Algorithm 1 as a numpy loop (update, then arg max; np.argmax returns the first maximum).

    ``euclid``: distances are np.sqrt of the FP32 squared distance (IEEE
    single-precision root, correctly rounded).
    """
    P = _as_xyz(xyz)
    n = P.shape[0]
    D = np.full(n, np.inf, dtype=np.float32)
    idx = np.empty(m, dtype=np.int32)
    d2 = np.empty(m, dtype=np.float32)
    idx[0], d2[0] = start, np.inf
    last = start
    for j in range(1, m):
        t = sqdist_np(P, P[last])
        if euclid:
            t = np.sqrt(t)
        np.minimum(D, t, out=D)   # equal values are bitwise identical, so min == strict update
        b = int(np.argmax(D))
        idx[j], d2[j] = b, D[b]
        last = b
    return idx, d2


def fps_bruteforce(xyz, m: int, start: int = 0, euclid: bool = False):
    """Selection rule of Sec. 3.1 from scratch: s_j = arg max_p min_{s in S_{j-1}} d(p, s).

    Every step recomputes the full point-to-chosen-set distance matrix (no
    incremental state), takes the row minimum, then the largest value with the
    smallest index.  Tiny clouds only.  ``euclid``: every squared distance is
    replaced by its correctly rounded root from ``sqrt_rn_exact``.
    """
    P = _as_xyz(xyz)
    chosen = [start]
    d2s = [np.float32(np.inf)]
    for _ in range(1, m):
        S = P[np.array(chosen)]
        d = P[:, None, :] - S[None, :, :]          # [n, |S|, 3] float32
        sq = d * d
        dist = (sq[..., 0] + sq[..., 1]) + sq[..., 2]
        if euclid:
            dist = _roots_exact(dist)
        near = dist.min(axis=1)
        best = near.max()
        bi = int(np.flatnonzero(near == best)[0])
        chosen.append(bi)
        d2s.append(best)
    return np.array(chosen, dtype=np.int32), np.array(d2s, dtype=np.float32)


def fps_exact_int(pts, m: int, start: int = 0):
    """The paper's Euclidean FPS on integer coordinates with exact integer arithmetic.

    The Euclidean norm is compared through its square, which orders exactly
    like the norm; all arithmetic is on Python integers, so no rounding occurs.
    Returns (idx list, squared distances list, -1 standing for +inf).
    """
    pts = [tuple(int(c) for c in p) for p in pts]
    n = len(pts)
    INF = None
    D = [INF] * n
    out, outd = [start], [-1]
    last = start
    for _ in range(1, m):
        sx, sy, sz = pts[last]
        for i, (x, y, z) in enumerate(pts):
            t = (x - sx) ** 2 + (y - sy) ** 2 + (z - sz) ** 2
            if D[i] is INF or t < D[i]:
                D[i] = t
        bi = max(range(n), key=lambda i: (D[i], -i))
        out.append(bi)
        outd.append(D[bi])
        last = bi
    return out, outd


def _roots_exact(a):
    """sqrt_rn_exact element-wise (each distinct value computed once)."""
    a = np.asarray(a, dtype=np.float32)
    u, inv = np.unique(a, return_inverse=True)
    r = np.array([sqrt_rn_exact(v) for v in u], dtype=np.float32)
    return r[inv].reshape(a.shape)


def sqrt_rn_exact(v) -> np.float32:
    """FP32 square root of a non-negative FP32 value, rounded to nearest, by integers.

    v = N * 4^q exactly with an integer N of at least 100 bits, so
    sqrt(v) = sqrt(N) * 2^q; the integer root s = isqrt(N) carries 50 or more
    bits, and rounding s (with the discarded fraction known to be non-zero
    unless s^2 = N) to 24 significant bits gives the correctly rounded root.
    """
    import math
    v = float(np.float32(v))
    if v == 0.0 or math.isinf(v):
        return np.float32(v)
    if not v > 0.0:
        raise ValueError("negative or NaN input")
    _, e = math.frexp(v)              # v = f * 2^e, 0.5 <= f < 1
    q = (e - 120) // 2                # 4^q well below v's last bit: N >= 2^119
    N = int(math.ldexp(v, -2 * q))    # exact: the scaled value is an integer
    assert math.ldexp(float(N), 2 * q) == v
    s = math.isqrt(N)
    inexact = s * s != N
    shift = s.bit_length() - 24
    t, rem = s >> shift, s & ((1 << shift) - 1)
    half = 1 << (shift - 1)
    # the true root is s + f with 0 <= f < 1 (f > 0 iff inexact)
    if rem > half or (rem == half and inexact) or (rem == half and not inexact and (t & 1)):
        t += 1
    return np.float32(math.ldexp(float(t), q + shift))
