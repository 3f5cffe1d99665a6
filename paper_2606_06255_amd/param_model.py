"""Voxel-parameter choice for RadiusFPS-G: the default rule and the trained network.

The paper sets the voxel resolution by hand and finds that the best value
depends on the cloud (Sec. 5.6.2).  Here a small network (include/rfps_mlp.h)
predicts, from 516 features of a cloud, how fast each of 36 candidate
(n_vox, shell spacing) pairs would run, and the cloud is indexed with the
predicted fastest one -- unless it is not predicted to beat the library's
default rule by a margin, in which case the default is kept.  No choice can
change the sampled sequence; it only changes the speed.

Everything on the GPU runs in librfps kernels: features, forward pass,
choice, and in training the gradient and Adam steps.  This module only
moves data and keeps the bookkeeping.

Training workflow (needs a GPU):
    python -m paper_2606_06255_amd.param_model --out DIR
generates clouds (half room-like, half LiDAR-like, N log-uniform in
[8000, 1048576], M = N // 4), times build + sample for every candidate on
every cloud (the sweep), trains the network on the training clouds and
evaluates its choices on held-out clouds and on the dense 1M-point LiDAR-like
cloud against the default rule and the best candidate of the sweep.

A sweep too long for one session is measured in slices and merged:
    python -m paper_2606_06255_amd.param_model --out DIR --part START COUNT
    python -m paper_2606_06255_amd.param_model --out DIR --merge PART.npz ...
    python -m paper_2606_06255_amd.param_model --out DIR --sweep DIR/sweep.npz
(cloud index total = train + held-out is the dense 1M-point cloud; every
slice regenerates its clouds from the seed, so slices are independent).
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import math
import os
import sys
import time

import numpy as np
import torch

from . import (MLP, MLP_CANDIDATES, MLP_INPUTS, MLP_OUTPUTS, MLP_PARAMS, F_TELEMETRY, build_index,
               default_n_vox, mlp_candidate, read_status, read_telemetry, sample)

_PKG = os.path.dirname(os.path.abspath(__file__))
MODEL_PATH = os.path.join(_PKG, "param_mlp.npz")
SHAPES = (("W1", (64, MLP_INPUTS)), ("b1", (64,)), ("W2", (64, 64)), ("b2", (64,)), ("W3", (MLP_OUTPUTS, 64)),
          ("b3", (MLP_OUTPUTS,)))


def candidates():
    return [mlp_candidate(k) for k in range(MLP_CANDIDATES)]


def default_candidate(n: int) -> int:
    """Candidate index of the library's default rule (its n_vox, one shell)."""
    nv = default_n_vox(n)
    for k, (cn, sh) in enumerate(candidates()):
        if cn == nv and sh == 0.0:
            return k
    raise ValueError("default n_vox %d is not a candidate" % nv)


def init_params(seed: int) -> np.ndarray:
    """He-uniform weights, zero biases (packed in the library's order)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W"):
            parts.append(rng.uniform(-1.0, 1.0, int(np.prod(shape))) * math.sqrt(6.0 / shape[1]))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    return np.concatenate(parts).astype(np.float32)


class ParamModel:
    """The trained network (weights from param_mlp.npz) on one device."""

    def __init__(self, device, path: str = MODEL_PATH, margin: float | None = None):
        data = np.load(path, allow_pickle=False)
        self.net = MLP(device)
        self.net.load(data["params"])
        self.margin = float(data["margin"]) if margin is None else float(margin)
        self.device = device
        self.feat = torch.empty(MLP_INPUTS, dtype=torch.float32, device=device)

    def choose(self, xyz: torch.Tensor):
        """(n_vox, shell spacing, candidate, predictions): waits for the device.
        A grid whose share per workgroup exceeds the on-chip budget makes
        the sampler report RFPS_ERR_CAPACITY; callers then index with the
        default rule (see fps_auto)."""
        n = xyz.shape[0]
        self.net.features(xyz, out=self.feat)
        k, y = self.net.choose(self.feat, default_candidate(n), self.margin)
        nv, sh = mlp_candidate(k)
        return nv, sh, k, y


def fitting_default(n: int, ms) -> int:
    """The default rule's candidate, or when its grid does not fit on chip
    (ms not finite) the next coarser one-shell grid that does (candidates
    run n_vox-major, the one-shell grid first)."""
    cand = candidates()
    d = default_candidate(n)
    while not np.isfinite(ms[d]) and d > 0:
        d -= 1
        while d > 0 and cand[d][1] != 0.0:
            d -= 1
    return d


def fps_auto(model: ParamModel, xyz: torch.Tensor, m: int, start: int = 0, **kw):
    """Exact FPS with the network's grid, falling back to the default rule
    (and then to coarser one-shell grids) when a grid does not fit on chip.
    Returns (idx, d2, (n_vox, shell))."""
    from . import RfpsError, fps
    nv, sh, _, _ = model.choose(xyz)
    grids = sorted({v for v, _ in candidates()}, reverse=True)
    tries = [(nv, sh)] + [(v, 0.0) for v in grids if v <= default_n_vox(xyz.shape[0])]
    for r, (v, s) in enumerate(tries):
        try:
            i, d = fps(xyz, m, start, n_vox=v, shell=s, **kw)
            return i, d, (v, s)
        except RfpsError as e:
            if e.status != 6 or r + 1 == len(tries):
                raise


# ---------------------------------------------------------------------------
# Sweep and training
# ---------------------------------------------------------------------------
def make_cloud(seed: int, i: int, n: int) -> np.ndarray:
    """Cloud i of a sweep: even i room-like, odd i LiDAR-like, n points."""
    import synth
    ss = np.random.SeedSequence([seed, i])
    if i % 2 == 0:
        return synth.room(ss, n=n)
    beams = 64 if n < 300_000 else 128
    steps = int(math.ceil(n / (beams * 0.995)))
    return synth.lidar(ss, beams=beams, azimuth_steps=steps, n_out=n)


def sweep_cloud(x: torch.Tensor, m: int, idx=None, repeats: int = 1, prune_rates: bool = True):
    """Build + sample time (ms, the median of `repeats` timed runs) and
    pruning rate (NaN unless prune_rates) of every candidate on one cloud,
    after one warm-up run of the default."""
    stream = torch.cuda.current_stream(x.device)
    n = x.shape[0]
    out_i = torch.empty(m, dtype=torch.int32, device=x.device)
    out_d = torch.empty(m, dtype=torch.float32, device=x.device)
    nv0 = default_n_vox(n)
    idx = build_index(x, n_vox=nv0, reuse=idx)
    sample(idx, m, 0, out_idx=out_i, out_d2=out_d)
    torch.cuda.synchronize()
    # every grid must give the same sequence; the reference is the first
    # that fits on chip (the default may not: its status is then 6)
    ref = out_i.clone() if read_status(idx) == 0 else None
    ms = np.zeros(MLP_CANDIDATES)
    prune = np.zeros(MLP_CANDIDATES)
    for k, (nv, sh) in enumerate(candidates()):
        # the time is the default (uninstrumented) sampler's; a second,
        # untimed call with telemetry gives the pruning rate
        times = []
        for _ in range(repeats):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            idx = build_index(x, n_vox=nv, shell=sh, reuse=idx)
            sample(idx, m, 0, out_idx=out_i, out_d2=out_d)
            b.record(stream)
            torch.cuda.synchronize()
            times.append(a.elapsed_time(b))
            if read_status(idx) != 0:
                break
        st = read_status(idx)
        if st == 0:
            if ref is None:
                ref = out_i.clone()
            if not torch.equal(out_i, ref):
                raise RuntimeError("candidate %d changed the sampled sequence" % k)
            if prune_rates:
                sample(idx, m, 0, flags=F_TELEMETRY, out_idx=out_i, out_d2=out_d)
                st = read_status(idx)
        if st == 6:
            # this grid's share per workgroup does not fit on chip: not a choice
            ms[k], prune[k] = np.nan, np.nan
            continue
        if st != 0:
            raise RuntimeError("candidate %d failed with status %d" % (k, st))
        if not torch.equal(out_i, ref):
            raise RuntimeError("candidate %d changed the sampled sequence" % k)
        ms[k] = float(np.median(times))
        if prune_rates:
            tel = read_telemetry(idx)
            prune[k] = 1.0 - tel["points_visited"] / max(1, tel["iters"] * n)
        else:
            prune[k] = np.nan
    return ms, prune, idx


def targets(ms, prune):
    """Network targets of one cloud: ln(ms_k) minus its mean over the
    candidates (the ranking is what matters), and the pruning rates.  A
    candidate that does not fit on chip gets the slowest time plus ln 2."""
    ok = np.isfinite(ms)
    lm = np.log(np.where(ok, ms, 1.0))
    lm[~ok] = lm[ok].max() + math.log(2.0)
    pr = np.where(np.isfinite(prune), prune, 0.0)
    return np.concatenate([lm - lm.mean(), pr]).astype(np.float32)


def train(X, T, device, steps=4000, lr=1e-3, seed=0, log=None, has_prune=None):
    """Full-batch Adam on the GPU with the library's training kernels."""
    net = MLP(device, rows=X.shape[0])
    net.load(init_params(seed))
    Xd = torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(device)
    Td = torch.from_numpy(np.ascontiguousarray(T, dtype=np.float32)).to(device)
    # the ranking head counts fully, the pruning-rate head a quarter (and not
    # at all for clouds swept without pruning rates)
    W = np.ones_like(T)
    W[:, MLP_CANDIDATES:] = 0.25
    if has_prune is not None:
        W[~np.asarray(has_prune), MLP_CANDIDATES:] = 0.0
    Wd = torch.from_numpy(W).to(device)
    loss = torch.empty(1, dtype=torch.float32, device=device)
    hist = []
    for s in range(steps):
        net.train_step(Xd, Td, Wd, lr=lr, loss=loss)
        if s % 500 == 0 or s == steps - 1:
            hist.append((s, float(loss.item())))
            if log:
                log("  step %d loss %.5f" % hist[-1])
    return net, hist


def evaluate(net, X, MS, N, margin):
    """Per cloud: time of the default, of the network's choice and of the
    sweep's best, from the measured sweep."""
    y = net.forward(torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to(net.device)).cpu().numpy()
    rows = []
    for b in range(X.shape[0]):
        d = fitting_default(int(N[b]), MS[b])
        pred = y[b, :MLP_CANDIDATES]
        k = int(np.argmin(pred))
        if not pred[k] < pred[d] - margin or not np.isfinite(MS[b, k]):
            k = d  # no clear predicted win, or a grid that does not fit: the default
        best = int(np.nanargmin(MS[b]))
        rows.append({"n": int(N[b]), "default": d, "choice": k, "best": best, "ms_default": float(MS[b, d]),
                     "ms_choice": float(MS[b, k]), "ms_best": float(MS[b, best])})
    gain = float(np.exp(np.mean([math.log(r["ms_default"] / r["ms_choice"]) for r in rows])))
    regret = float(np.exp(np.mean([math.log(r["ms_choice"] / r["ms_best"]) for r in rows])))
    headroom = float(np.exp(np.mean([math.log(r["ms_default"] / r["ms_best"]) for r in rows])))
    return {"gain_vs_default": gain, "regret_vs_best": regret, "best_vs_default": headroom, "clouds": rows}


def report_markdown(report: dict, command: str) -> str:
    """The evaluation as a markdown summary (held-out clouds listed one by one)."""
    def grid(k):
        nv, sh = mlp_candidate(k)
        return "n_vox %d, %s" % (nv, "one shell" if sh == 0.0 else "%g m" % sh)

    out = ["# Voxel-parameter network: evaluation on held-out clouds", "",
           "Sweep, training and evaluation by `paper_2606_06255_amd/param_model.py` on one MI355X.",
           "Every time is the median of %d timed runs of build + sample (M = N/4; M = 65,536 for the dense"
           % report["repeats"],
           "LiDAR cloud) with the given grid and the library's default sampler settings, HIP events, after a",
           "warm-up run; every grid was checked to give the same selections as the first grid that fits on chip.",
           "A default grid that does not fit counts as the next coarser one-shell grid that does.", "",
           "Command (from the repository root on the GPU host):", "", "```", command, "```", "",
           "Training: %d clouds, full-batch Adam on the GPU (library kernels), %d steps, lr %g; choice margin "
           "%g (log units). Final training loss %.4f." % (report["train_clouds"], report["steps"], report["lr"],
                                                         report["margin"], report["loss"][-1][1]), "",
           "Gains are geometric means over clouds of time(default rule) / time(choice); 'best' is the",
           "fastest of the 36 measured grids (the grid search), so best/default is the headroom.", "",
           "| set | clouds | network vs default | network regret vs best | best vs default |",
           "|---|---:|---:|---:|---:|"]
    names = {"train": "training clouds", "heldout": "held-out clouds", "dense_lidar_1M": "dense LiDAR, N = 1,048,576"}
    for k in ("train", "heldout", "dense_lidar_1M"):
        r = report[k]
        out.append("| %s | %d | %.3fx | %.3fx | %.3fx |" % (names[k], len(r["clouds"]), r["gain_vs_default"],
                                                         r["regret_vs_best"], r["best_vs_default"]))
    c = report["dense_lidar_1M"]["clouds"][0]
    out += ["", "Dense LiDAR cloud: default %s %.2f ms; network %s %.2f ms; best %s %.2f ms." % (
        grid(c["default"]), c["ms_default"], grid(c["choice"]), c["ms_choice"], grid(c["best"]), c["ms_best"]),
        "", "Held-out clouds:", "", "| N | default | ms | network choice | ms | best ms |", "|---:|---|---:|---|---:|---:|"]
    for c in report["heldout"]["clouds"]:
        out.append("| %d | %s | %.2f | %s | %.2f | %.2f |" % (c["n"], grid(c["default"]), c["ms_default"],
                                                             grid(c["choice"]), c["ms_choice"], c["ms_best"]))
    return "\n".join(out) + "\n"


def cloud_sizes(seed: int, total: int, n_min: int, n_max: int) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return np.floor(np.exp(rng.uniform(math.log(n_min), math.log(n_max), total))).astype(np.int64)


def sweep_range(args, start: int, count: int, dev, log, save=None):
    """Sweeps clouds [start, start + count) of the set (index total = the
    dense 1M-point cloud); cloud generation runs ahead on host threads.
    save(X, MS, PR, N, I) is called every 25 clouds with what is done."""
    import synth
    total = args.train_clouds + args.heldout_clouds
    sizes = cloud_sizes(args.seed, total, args.n_min, args.n_max)
    ids = list(range(start, min(start + count, total + 1)))

    def gen(i):
        if i < total:
            n = int(sizes[i])
            return make_cloud(args.seed, i, n), n // 4
        P = synth.dense_lidar(0)
        return P, 65536

    net = MLP(dev)
    X = np.zeros((len(ids), MLP_INPUTS), dtype=np.float32)
    MS = np.zeros((len(ids), MLP_CANDIDATES))
    PR = np.zeros((len(ids), MLP_CANDIDATES))
    N = np.zeros(len(ids), dtype=np.int64)
    idx = None
    t0 = time.time()
    with cf.ThreadPoolExecutor(max_workers=4) as ex:
        futs = [ex.submit(gen, i) for i in ids[:4]]
        for r, i in enumerate(ids):
            P, m = futs[r].result()
            if r + 4 < len(ids):
                futs.append(ex.submit(gen, ids[r + 4]))
            n = P.shape[0]
            x = torch.from_numpy(P).to(dev)
            X[r] = net.features(x).cpu().numpy()
            # pruning rates are a secondary training target: every
            # args.prune_every-th training cloud (and the dense cloud)
            MS[r], PR[r], idx = sweep_cloud(x, m, idx, repeats=args.repeats,
                                            prune_rates=(i < args.train_clouds and i % args.prune_every == 0)
                                            or i == total)
            N[r] = n
            log("cloud %d (%d/%d) N=%d M=%d default %.2f ms best %.2f ms (cand %d) worst %.2f ms, %d unfit  [%.0f s]" % (
                i, r + 1, len(ids), n, m, MS[r, default_candidate(n)], np.nanmin(MS[r]), int(np.nanargmin(MS[r])),
                np.nanmax(MS[r]), int(np.isnan(MS[r]).sum()), time.time() - t0))
            if save is not None and (r % 25 == 24 or r == len(ids) - 1):
                save(X[:r + 1], MS[:r + 1], PR[:r + 1], N[:r + 1], np.array(ids[:r + 1], dtype=np.int64))
    return X, MS, PR, N, np.array(ids, dtype=np.int64)


def main(argv=None):
    ap = argparse.ArgumentParser(description="sweep, train and evaluate the voxel-parameter network")
    ap.add_argument("--out", required=True)
    ap.add_argument("--train-clouds", type=int, default=2000)
    ap.add_argument("--heldout-clouds", type=int, default=200)
    ap.add_argument("--n-min", type=int, default=8000)
    ap.add_argument("--n-max", type=int, default=1 << 20)
    ap.add_argument("--repeats", type=int, default=3, help="timed runs per candidate (median)")
    ap.add_argument("--prune-every", type=int, default=4,
                    help="measure pruning rates on every n-th training cloud (a second, instrumented run)")
    ap.add_argument("--steps", type=int, default=4000)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--margin", type=float, default=0.03)
    ap.add_argument("--seed", type=int, default=2606)
    ap.add_argument("--sweep", default="", help="train on a saved sweep (npz) instead of measuring")
    ap.add_argument("--part", type=int, nargs=2, metavar=("START", "COUNT"),
                    help="only sweep clouds [START, START + COUNT) and save them as a part")
    ap.add_argument("--merge", nargs="+", default=None, help="merge saved parts into OUT/sweep.npz and stop")
    args = ap.parse_args(argv)
    os.makedirs(args.out, exist_ok=True)

    def log(*a):
        print(*a, flush=True)

    total = args.train_clouds + args.heldout_clouds
    if args.merge:
        parts = [np.load(f, allow_pickle=False) for f in args.merge]
        I = np.concatenate([d["I"] for d in parts])
        order = np.argsort(I)
        if not np.array_equal(I[order], np.arange(total + 1)):
            raise SystemExit("parts do not cover clouds 0..%d exactly once" % total)
        out = {k: np.concatenate([d[k] for d in parts])[order] for k in ("X", "MS", "PR", "N")}
        np.savez_compressed(os.path.join(args.out, "sweep.npz"), I=I[order], **out)
        log("merged %d clouds into %s" % (I.size, os.path.join(args.out, "sweep.npz")))
        return 0

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.part:
        start, count = args.part
        path = os.path.join(args.out, "sweep_part_%05d.npz" % start)

        def save(X, MS, PR, N, I):
            np.savez(path + ".tmp.npz", X=X, MS=MS, PR=PR, N=N, I=I)
            os.replace(path + ".tmp.npz", path)

        sweep_range(args, start, count, dev, log, save=save)
        log("saved %s" % path)
        return 0
    if args.sweep:
        d = np.load(args.sweep, allow_pickle=False)
        X, MS, PR, N = d["X"], d["MS"], d["PR"], d["N"]
        if X.shape[0] != total + 1:
            raise SystemExit("the sweep holds %d clouds, expected %d" % (X.shape[0], total + 1))
    else:
        X, MS, PR, N, _ = sweep_range(args, 0, total + 1, dev, log)
        np.savez(os.path.join(args.out, "sweep.npz"), X=X, MS=MS, PR=PR, N=N, I=np.arange(total + 1))
    ntr = args.train_clouds
    T = np.stack([targets(MS[i], PR[i]) for i in range(X.shape[0])])
    has_prune = np.isfinite(PR).any(axis=1)
    log("training on %d clouds" % ntr)
    net, hist = train(X[:ntr], T[:ntr], dev, steps=args.steps, lr=args.lr, seed=args.seed, log=log,
                      has_prune=has_prune[:ntr])
    params = net.save()
    report = {"train": evaluate(net, X[:ntr], MS[:ntr], N[:ntr], args.margin),
              "heldout": evaluate(net, X[ntr:-1], MS[ntr:-1], N[ntr:-1], args.margin),
              "dense_lidar_1M": evaluate(net, X[-1:], MS[-1:], N[-1:], args.margin),
              "loss": hist, "margin": args.margin, "train_clouds": ntr, "heldout_clouds": int(X.shape[0] - ntr - 1),
              "steps": args.steps, "lr": args.lr, "seed": args.seed, "repeats": args.repeats}
    for k in ("train", "heldout", "dense_lidar_1M"):
        r = report[k]
        log("%s: gain vs default %.3fx, regret vs best %.3fx, best vs default %.3fx" % (
            k, r["gain_vs_default"], r["regret_vs_best"], r["best_vs_default"]))
    np.savez(os.path.join(args.out, "param_mlp.npz"), params=params, margin=np.float32(args.margin))
    with open(os.path.join(args.out, "param_report.json"), "w") as f:
        json.dump(report, f, indent=1)
    with open(os.path.join(args.out, "param_model_evaluation.md"), "w") as f:
        f.write(report_markdown(report, "python3 -m paper_2606_06255_amd.param_model " + " ".join(
            sys.argv[1:] if argv is None else argv)))
    return 0


if __name__ == "__main__":
    sys.exit(main())
