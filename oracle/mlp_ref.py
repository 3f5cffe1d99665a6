"""ORACLE -- test infrastructure, not product code.

Only the tests, the smoke check and the benchmark's CPU-baseline leg may
import this module.  It shares no code with the device path.

Plain FP64 reference of the voxel-parameter network: cloud features, the
forward pass, the loss, its gradient and one Adam step, written from their
definitions.  The paper has no learned component (it tunes the voxel count by
hand, Sec. 5.6.2), so this module is "parity unpinned" with
respect to the paper: it is pinned instead by central finite differences of
its own loss, by closed forms of the Adam step and the bf16 rounding, and by
brute-force feature counts (tests/test_mlp_ref.py).

Network: 516 inputs -> 64 (ReLU) -> 64 (ReLU) -> 72 outputs.  Weight
matrices are stored in bfloat16 (round to nearest even of the FP32 master
copy) and used as such in the forward pass; biases stay FP32.  Gradients
with respect to the master weights are those of the rounded weights (the
rounding passes gradients straight through).
"""
from __future__ import annotations

import numpy as np

F_IN, H1, H2 = 516, 64, 64
N_VOX_CAND = (12, 16, 24, 32, 48, 64, 96, 128, 192)
SHELL_CAND = (0.0, 5.0, 10.0, 20.0)        # 0 = one shell (the uniform grid)
N_CAND = len(N_VOX_CAND) * len(SHELL_CAND)  # 36
OUT = 2 * N_CAND                            # log-ms and pruning rate per candidate
SHAPES = (("W1", (H1, F_IN)), ("b1", (H1,)), ("W2", (H2, H1)), ("b2", (H2,)), ("W3", (OUT, H2)),
          ("b3", (OUT,)))
N_PARAMS = sum(int(np.prod(s)) for _, s in SHAPES)


def candidate(k: int):
    """(n_vox, shell spacing) of candidate k: n_vox major, shells minor."""
    return N_VOX_CAND[k // len(SHELL_CAND)], SHELL_CAND[k % len(SHELL_CAND)]


def unpack(theta):
    """Views of the packed parameter vector, in SHAPES order."""
    out, o = {}, 0
    for name, shape in SHAPES:
        size = int(np.prod(shape))
        out[name] = theta[o:o + size].reshape(shape)
        o += size
    return out


def bf16_round(x):
    """FP32 value of bfloat16(float32(x)), round to nearest, ties to even."""
    u = np.ascontiguousarray(np.asarray(x, dtype=np.float32)).view(np.uint32).astype(np.uint64)
    lsb = (u >> np.uint64(16)) & np.uint64(1)
    r = ((u + np.uint64(0x7FFF) + lsb) & np.uint64(0xFFFF0000)).astype(np.uint32)
    return r.view(np.float32).astype(np.float64)


def features(xyz):
    """516 features of a cloud: (ln N - 11) / 2, ln(1 + E_a) / 2 for the
    three bounding-box extents, and ln(1 + 64 * count / N) for the 8^3 cells
    of a cubic grid over the box (cell edge (1 + 1e-4) * max(E) / 8, FP64
    coordinates, clamped).  Returned as float32, with the integer counts."""
    p = np.asarray(xyz, dtype=np.float32).astype(np.float64)
    n = p.shape[0]
    lo, hi = p.min(axis=0), p.max(axis=0)
    E = hi - lo
    emax = E.max()
    edge = (1.0 + 1e-4) * emax / 8.0 if emax > 0 else 1.0
    b = np.floor((p - lo[None, :]) / edge)
    b = np.clip(b, 0, 7).astype(np.int64)
    cell = (b[:, 2] * 8 + b[:, 1]) * 8 + b[:, 0]
    counts = np.bincount(cell, minlength=512).astype(np.float64)
    f = np.empty(F_IN, dtype=np.float64)
    f[0] = (np.log(float(n)) - 11.0) / 2.0
    f[1:4] = np.log1p(E) / 2.0
    f[4:] = np.log1p(64.0 * counts / n)
    return f.astype(np.float32), counts.astype(np.int64)


def forward(theta, X, quantize=True):
    """Outputs [B, 72] and the intermediate values, all FP64.  With
    quantize=False the weights are used unrounded (for derivative checks)."""
    P = unpack(np.asarray(theta, dtype=np.float64))
    q = bf16_round if quantize else (lambda w: np.asarray(w, dtype=np.float64))
    W1, W2, W3 = q(P["W1"]), q(P["W2"]), q(P["W3"])
    if quantize:
        b1, b2, b3 = (np.asarray(P[k], dtype=np.float32).astype(np.float64) for k in ("b1", "b2", "b3"))
    else:
        b1, b2, b3 = P["b1"], P["b2"], P["b3"]
    X = np.asarray(X, dtype=np.float32).astype(np.float64)
    Z1 = X @ W1.T + b1
    A1 = np.maximum(Z1, 0.0)
    Z2 = A1 @ W2.T + b2
    A2 = np.maximum(Z2, 0.0)
    Y = A2 @ W3.T + b3
    return Y, (X, Z1, A1, Z2, A2, W1, W2, W3)


def loss(theta, X, T, Wt, quantize=True):
    """Weighted squared error, sum over outputs, mean over the batch."""
    Y, _ = forward(theta, X, quantize)
    T = np.asarray(T, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    return float(np.sum(Wt * (Y - T) ** 2) / X.shape[0])


def gradient(theta, X, T, Wt, quantize=True):
    """d loss / d theta (packed like theta) and the loss, by the chain rule."""
    Y, (Xd, Z1, A1, Z2, A2, W1, W2, W3) = forward(theta, X, quantize)
    B = Xd.shape[0]
    T = np.asarray(T, dtype=np.float64)
    Wt = np.asarray(Wt, dtype=np.float64)
    dY = 2.0 * Wt * (Y - T) / B
    g = {}
    g["W3"] = dY.T @ A2
    g["b3"] = dY.sum(axis=0)
    dA2 = dY @ W3
    dZ2 = dA2 * (Z2 > 0)
    g["W2"] = dZ2.T @ A1
    g["b2"] = dZ2.sum(axis=0)
    dA1 = dZ2 @ W2
    dZ1 = dA1 * (Z1 > 0)
    g["W1"] = dZ1.T @ Xd
    g["b1"] = dZ1.sum(axis=0)
    flat = np.concatenate([g[name].ravel() for name, _ in SHAPES])
    return flat, float(np.sum(Wt * (Y - T) ** 2) / B)


def adam(theta, m, v, g, step, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam step (bias-corrected moments) on the FP64 master vector;
    `step` counts from 1."""
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    mh = m / (1.0 - beta1 ** step)
    vh = v / (1.0 - beta2 ** step)
    return theta - lr * mh / (np.sqrt(vh) + eps), m, v
