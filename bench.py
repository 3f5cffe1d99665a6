#!/usr/bin/env python3
"""Benchmark of the RadiusFPS-G hot path on one MI355X.

Default workload: the dense LiDAR-like cloud (128 beams x 8192 azimuth steps,
N = 1,048,576 points, FP32) sampled to M = 65,536 points with exact FPS.
One step = the whole path on one cloud already resident in HBM: voxel
parameter choice, index build (bounding box, voxel ids, radix sort, gather,
compaction, tiles and spheres) and the persistent sampler (all M selections).

With --workload batch one step is one batched call (index build and
sampling of 32 uneven clouds in one persistent launch, parameters from the
library's autotuner, picked during warm-up), replayed from a captured HIP
graph; per-cloud launches of the single-cloud path, the batched call
without the graph and per-cloud plain FPS are timed beside it.

Prints one JSON line (rank 0).  `value` is selected points per second over
the timed steps; `ms_per_step` is the ms per cloud.  Beside it: the plain GPU
FPS comparators on the same cloud and GPU, the roofline of the sampler kernel
(algorithmic bytes / measured kernel time vs the 8 TB/s HBM peak) and the
CPU oracle on the host cores (`cpu_baseline`, a bounded prefix of the run).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "ms per cloud & selected pts/s, RadiusFPS-G vs plain FPS, bit-exact indices"
HBM_PEAK_GBS = 8000.0
# LDS: 256 compute units x 128 bytes per clock x 2.4 GHz (the per-CU LDS rate
# of CDNA3, taken as the floor for gfx950)
LDS_PEAK_GBS = 256 * 128 * 2.4
PHASES = ("lookahead", "lookahead_copy", "lookahead_select", "exchange", "exchange_poll", "exchange_keys",
          "wait", "merge", "merge_list", "merge_rank", "merge_walk", "merge_picks", "apply", "apply_loop",
          "apply_update")
WORKLOADS = {
    "dense_lidar": "dense LiDAR-like cloud, 128 beams x 8192 azimuth, N=1,048,576, M=65,536",
    "room": "indoor room-like cloud, N=80,000, M=20,000",
    "lidar": "spinning LiDAR-like cloud, 64 beams x 1800 azimuth minus 576 drops, N=114,624, M=28,656",
    "cube": "uniform unit cube, N=4096, M=1024",
    "lidar_stages": "spinning LiDAR-like cloud, N=114,624, FPS in three stages 114,624 -> 28,656 -> 7,164 -> "
                    "1,791, each stage sampling the previous stage's picks in pick order",
    "batch": "32 uneven clouds in one call, N_i log-uniform in [8000, 120000], even i room-like, odd i "
             "LiDAR-like, M_i = N_i // 4, int32 CSR offsets",
}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def load_workload(name):
    import synth
    if name == "dense_lidar":
        return synth.dense_lidar(0), 65536
    if name == "room":
        return synth.room(0), 20000
    if name == "lidar":
        return synth.lidar(0), 28656
    if name == "cube":
        return synth.cube(0), 1024
    raise SystemExit("unknown workload " + name)


def source_digest():
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2606_06255_amd", "csrc")
    for f in sorted(os.listdir(csrc)):
        if f.endswith((".hip", ".h")):
            h.update(open(os.path.join(csrc, f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic(workload, digest):
    """HBM traffic per sampler launch measured with rocprofv3 counters, if the
    kernels have not changed since (profiles/traffic.json, keyed by source digest)."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    try:
        rec = json.load(open(path)).get(workload)
    except (OSError, ValueError):
        return None
    if not rec or rec.get("source_digest") != digest:
        return None
    return rec.get("bytes_per_launch")


def main():
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="dense_lidar", choices=sorted(WORKLOADS))
    ap.add_argument("--n-vox", type=int, default=0, help="voxel bins per axis (0 = library default)")
    ap.add_argument("--groups", type=int, default=0, help="sampler workgroups (0 = one per CU)")
    ap.add_argument("--lookahead", type=int, default=0, help="candidates per workgroup per round (0 = default)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-comparators", action="store_true")
    ap.add_argument("--copy-mb", type=int, default=256, help="size of the copy kernel used to calibrate counters")
    ap.add_argument("--cpu-seconds", type=float, default=12.0, help="CPU time budget of the oracle baseline")
    ap.add_argument("--ablation", action="store_true",
                    help="also time the sampler variants of the paper's ablation (pruning, point skip, one "
                         "persistent kernel vs two launches per selection) on the same index")
    ap.add_argument("--cpu-sweep", action="store_true",
                    help="also time the CPU RadiusFPS entry point for every voxel resolution of the default "
                         "rule's candidate list, one thread and the default team (the sensitivity to v of Sec. 5.6.2)")
    ap.add_argument("--distance", default="squared", choices=("squared", "euclid"),
                    help="FPS over FP32 squared distances (default) or over their rounded roots (RFPS_F_SQRT); "
                         "euclid is available for the single-cloud workloads")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (batched clouds would shard "
              "across GPUs by cost with no exchange; a single cloud needs one exchange per round)",
              file=sys.stderr)
        return 2
    if args.distance == "euclid" and args.workload in ("batch", "lidar_stages"):
        print("--distance euclid is available for the single-cloud workloads", file=sys.stderr)
        return 2

    import numpy as np
    import torch

    import paper_2606_06255_amd as rf

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        return 1
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    stream = torch.cuda.current_stream(dev)

    if args.workload == "batch":
        result = run_batch(args, rf, dev, stream)
        print(json.dumps(result), flush=True)
        return 0
    if args.workload == "lidar_stages":
        result = run_stages(args, rf, dev, stream)
        print(json.dumps(result), flush=True)
        return 0

    P, M = load_workload(args.workload)
    N = P.shape[0]
    x = torch.from_numpy(P).to(dev)
    n_vox = args.n_vox or rf.default_n_vox(N)
    out_i = torch.empty(M, dtype=torch.int32, device=dev)
    out_d = torch.empty(M, dtype=torch.float32, device=dev)
    idx = rf.build_index(x, n_vox=n_vox)
    euclid = args.distance == "euclid"
    fdist = rf.F_SQRT if euclid else 0

    def step(with_sample_events=None):
        nonlocal idx
        idx = rf.build_index(x, n_vox=n_vox, reuse=idx)
        if with_sample_events is not None:
            with_sample_events[0].record(stream)
        rf.sample(idx, M, 0, groups=args.groups, lookahead=args.lookahead, flags=fdist, out_idx=out_i,
                  out_d2=out_d)
        if with_sample_events is not None:
            with_sample_events[1].record(stream)

    # ---- timed region -------------------------------------------------------
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    st = rf.read_status(idx)
    if st != 0:
        raise rf.RfpsError(st, "device status")
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(args.steps)]
    sev = [torch.cuda.Event(enable_timing=True) for _ in range(args.steps + 1)]  # step boundaries
    t_all0, t_all1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t_all0.record(stream)
    sev[0].record(stream)
    for k in range(args.steps):
        step(ev[k])
        sev[k + 1].record(stream)
    t_all1.record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    total_ms = t_all0.elapsed_time(t_all1)
    sample_ms = [a.elapsed_time(b) for a, b in ev]
    step_ms = [sev[k].elapsed_time(sev[k + 1]) for k in range(args.steps)]
    ms_per_step = total_ms / args.steps
    st = rf.read_status(idx)
    if st != 0:
        raise rf.RfpsError(st, "device status")
    got_i = out_i.cpu().numpy().copy()
    got_d = out_d.cpu().numpy().copy()
    log("timed %d steps: %.3f ms/step (wall %.3f ms/step), sampler %.3f ms" %
        (args.steps, ms_per_step, 1e3 * (wall1 - wall0) / args.steps, float(np.mean(sample_ms))))

    # ---- untimed: build time, telemetry, trace ------------------------------
    b0, b1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    b0.record(stream)
    idx = rf.build_index(x, n_vox=n_vox, reuse=idx)
    b1.record(stream)
    torch.cuda.synchronize()
    build_ms = b0.elapsed_time(b1)
    info = rf.read_index_info(idx)
    rf.sample(idx, M, 0, groups=args.groups, lookahead=args.lookahead, flags=rf.F_TELEMETRY | rf.F_TRACE | fdist,
              out_idx=out_i, out_d2=out_d)
    tel = rf.read_telemetry(idx)
    tr, hz = rf.read_trace(idx)
    lookahead = args.lookahead or 2
    # phase clocks of workgroup 0 without the counters (instrumented kernel)
    idx = rf.build_index(x, n_vox=n_vox, reuse=idx)
    rf.sample(idx, M, 0, groups=args.groups, lookahead=args.lookahead, flags=rf.F_CLOCKS | fdist, out_idx=out_i,
              out_d2=out_d)
    clk = rf.read_telemetry(idx)
    nr = max(1, clk["exchanges"])
    phases = {k: clk["ticks_" + k] / clk["tick_hz"] / nr * 1e6 for k in PHASES}
    phases["lookahead_update"] = phases["lookahead"] - phases["lookahead_copy"] - phases["lookahead_select"]
    phases["round"] = sum(phases[k] for k in ("lookahead", "exchange", "merge", "apply"))
    merge_stats = {"above": clk["merge_above"] / nr, "listed": clk["merge_listed"] / nr,
                   "failures": clk["merge_failures"] / nr, "wg0_apply_pairs": clk["apply_pairs"] / nr,
                   "wg0_apply_rekeys": clk["apply_rekeys"] / nr}
    # latency floor of one exchange round: bare exchanges of the sampler's
    # slot size among the same workgroups (nothing else in the round)
    G_used = args.groups or 0
    ex_floor_us = rf.probe_exchange(idx, words=6 * lookahead + 2, rounds=2000, groups=G_used)
    ex_floor_1w_us = rf.probe_exchange(idx, words=1, rounds=2000, groups=G_used)
    # per exchange round: (publish time, outcome time | picks << 48)
    picks_per_round = (tr[:, 1] >> np.uint64(48)).astype(np.int64)
    t_done = (tr[:, 1] & np.uint64((1 << 48) - 1)).astype(np.int64)
    ex_us = (t_done - tr[:, 0].astype(np.int64)).astype(np.float64) / hz * 1e6
    it_us = np.diff(t_done) / hz * 1e6 if len(t_done) > 1 else np.zeros(1)
    NT = info["n_tiles"]
    # algorithmic bytes of one sampler launch:
    #   prologue: 16 B per point (x, y, z, original index) + 20 B per tile (sphere, count)
    #   per update round: 24 B per tile (sphere test 16 B + key scan 8 B),
    #     16 B per visited point (x, y, z, D), 4 B per updated D, 12 B per resynced tile
    #   per selection: 8 B of output
    alg_bytes = (16 * N + 20 * NT + 24 * NT * tel["iters"] + 16 * tel["points_visited"]
                 + 4 * tel["points_updated"] + 12 * tel["tiles_resynced"] + 8 * (M - 1))
    samp_s = float(np.mean(sample_ms)) / 1e3
    achieved = alg_bytes / samp_s / 1e9
    digest = source_digest()
    traffic = None if euclid else stored_traffic(args.workload, digest)
    pruned_frac = 1.0 - tel["points_visited"] / max(1, tel["iters"] * N)
    rounds = int(len(tr))
    lat_floor_ms = rounds * ex_floor_us / 1e3
    fr = {"hbm_algorithmic": achieved / HBM_PEAK_GBS, "lds": achieved / LDS_PEAK_GBS,
          "latency": lat_floor_ms / (samp_s * 1e3)}
    if traffic is not None:
        fr["hbm_counted"] = traffic / samp_s / 1e9 / HBM_PEAK_GBS
    # what binds: the algorithmic bytes are served from LDS, so against HBM
    # they measure work per unit time, not a bound; the bounds compared are
    # the LDS peak, the counted HBM traffic and the exchange latency floor
    bound = max((k for k in fr if k != "hbm_algorithmic"), key=fr.get).split("_")[0]

    result = {
        "metric": METRIC,
        "value": M / (ms_per_step / 1e3),
        "unit": "selected pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": args.workload, "description": WORKLOADS[args.workload], "n_points": N,
                   "m": M, "start": 0, "n_vox": n_vox, "tile": 64, "lookahead": args.lookahead or 2,
                   "distance": args.distance,
                   "groups": args.groups or (torch.cuda.get_device_properties(dev).multi_processor_count //
                                             (1 if N >= 65536 else 2))},
        "ms_per_cloud": ms_per_step,
        "step_ms_percentiles": {"p10": float(np.percentile(step_ms, 10)), "p50": float(np.median(step_ms)),
                                "p90": float(np.percentile(step_ms, 90))},
        "build_ms": build_ms,
        "sample_ms": float(np.mean(sample_ms)),
        "index": {"voxels": info["n_voxels"], "tiles": NT},
        "pruning": {"point_visit_fraction": 1.0 - pruned_frac, "pruned_fraction": pruned_frac,
                    "tiles_pruned_fraction": tel["tiles_pruned"] / max(1, tel["tile_tests"]), **tel},
        "exchange_rounds": rounds,
        "selections_per_round": float((M - 1) / max(1, len(tr))),
        "exchange_us": {"p10": float(np.percentile(ex_us, 10)), "p50": float(np.percentile(ex_us, 50)),
                        "p90": float(np.percentile(ex_us, 90)), "round_p50": float(np.median(it_us)),
                        "note": "publish to merged outcome of workgroup 0, per exchange round"},
        "round_phases_us": phases,
        "merge_per_round": merge_stats,
        "exchange_floor_us": {"slot_words": 6 * lookahead + 2, "per_round": ex_floor_us,
                              "one_word_per_round": ex_floor_1w_us,
                              "note": "bare exchange rounds (publish, read every slot) among the same workgroups"},
        "latency_floor_ms": lat_floor_ms,
        # the sampler keeps its state in LDS and waits on one exchange per
        # round: it is latency-bound.  achieved / peak / frac are the
        # algorithmic bytes of a launch over its time against the HBM peak;
        # `fractions` sets them beside the LDS peak, the counted HBM bytes and
        # the exchange latency floor (rounds x bare exchange round), and
        # `bound` names the largest of the last three.
        "roofline": {"bound": bound, "kernel":
                     "k_rfps_rounds%s<%d>" % ("_euclid" if euclid else "", lookahead),
                     "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": traffic, "fractions": fr, "lds_peak_gbs": LDS_PEAK_GBS,
                     "alg_bytes_per_launch": alg_bytes,
                     "alg_bytes_per_selection": alg_bytes / max(1, M - 1), "source_digest": digest},
    }

    # ---- comparators (untimed region, same cloud, same GPU) ----------------
    if not args.no_comparators and euclid:
        # the plain kernels sample squared distances only; the ablation is the
        # same sampler with one selection per exchange
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rf.sample(idx, M, 0, groups=args.groups, flags=rf.F_SINGLE_PICK | fdist, out_idx=out_i, out_d2=out_d)
        b.record(stream)
        torch.cuda.synchronize()
        result["comparators"] = {"rfps_single_pick_sample_ms": a.elapsed_time(b)}
        result["bitexact_vs_single_pick"] = bool(np.array_equal(out_i.cpu().numpy(), got_i) and np.array_equal(
            out_d.cpu().numpy().view(np.uint32), got_d.view(np.uint32)))
    elif not args.no_comparators:
        ws = rf.PlainWorkspace(N, dev)
        best = None
        comps = {}
        for g in (0, 128, 192, 256):
            try:
                rf.fps_plain(x, M, 0, variant=0, groups=g, ws=ws, out_idx=out_i, out_d2=out_d)
            except rf.RfpsError:
                continue
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            rf.fps_plain(x, M, 0, variant=0, groups=g, ws=ws, out_idx=out_i, out_d2=out_d, check=False)
            b.record(stream)
            torch.cuda.synchronize()
            t = a.elapsed_time(b)
            comps["plain_persistent_g%d_ms" % g] = t
            if best is None or t < best[0]:
                best = (t, g, out_i.cpu().numpy().copy(), out_d.cpu().numpy().copy())
        same = best is not None and np.array_equal(best[2], got_i) and np.array_equal(
            best[3].view(np.uint32), got_d.view(np.uint32))
        mm = min(M, 2000)
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rf.fps_plain(x, mm, 0, variant=1, ws=ws, out_idx=out_i, out_d2=out_d)
        b.record(stream)
        torch.cuda.synchronize()
        one_wg_ms = a.elapsed_time(b) * (M - 1) / (mm - 1)
        same_1wg = np.array_equal(out_i.cpu().numpy()[:mm], got_i[:mm])
        # ablation: the same sampler with one selection per exchange
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        rf.sample(idx, M, 0, groups=args.groups, flags=rf.F_SINGLE_PICK, out_idx=out_i, out_d2=out_d)
        b.record(stream)
        torch.cuda.synchronize()
        single_ms = a.elapsed_time(b)
        same_single = np.array_equal(out_i.cpu().numpy(), got_i)
        result["comparators"] = {
            "rfps_single_pick_sample_ms": single_ms,
            "plain_persistent_best_ms": best[0] if best else None,
            "plain_persistent_best_groups": best[1] if best else None,
            "plain_one_workgroup_ms": one_wg_ms,
            "plain_one_workgroup_note": "timed on the first %d selections; per-selection cost is constant" % mm,
            **comps,
        }
        result["speedup_vs_plain_persistent"] = (best[0] / ms_per_step) if best else None
        result["speedup_vs_plain_one_workgroup"] = one_wg_ms / ms_per_step
        result["bitexact_vs_plain"] = bool(same and same_1wg and same_single)

    if args.ablation:
        result["ablation"] = run_ablation(rf, idx, M, fdist, got_i, got_d, stream, torch, np)

    # ---- counter calibration: a plain copy of known size ---------------------
    nbytes = args.copy_mb << 20
    src = torch.empty(nbytes // 4, dtype=torch.float32, device=dev).fill_(1.0)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    result["copy_calibration_bytes"] = nbytes

    # ---- CPU baseline: the oracle on the host cores, bounded prefix ---------
    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline([P], [M], [got_i], [got_d], args.cpu_seconds, euclid=euclid)
        result["cpu_radiusfps"] = cpu_product(rf, P, M, fdist, got_i, got_d, np)
    if args.cpu_sweep:
        result["cpu_vox_sweep"] = cpu_vox_sweep(rf, P, M, fdist, got_i, np)

    print(json.dumps(result), flush=True)
    return 0


def cpu_product(rf, P, M, fdist, got_i, got_d, np):
    """The library's CPU RadiusFPS (rfps_cpu_sample, host cores, default
    team) on the whole workload, and one thread on a prefix of it."""
    t0 = time.perf_counter()
    ci, cd = rf.cpu_fps(P, M, 0, flags=fdist)
    dt = time.perf_counter() - t0
    same = bool(np.array_equal(ci, got_i) and np.array_equal(cd.view(np.uint32), got_d.view(np.uint32)))
    mp = min(M, 4096)
    t0 = time.perf_counter()
    si, _ = rf.cpu_fps(P, mp, 0, flags=fdist, threads=1)
    dt1 = time.perf_counter() - t0
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or len(os.sched_getaffinity(0))
    return {"value": (M - 1) / dt, "unit": "selected pts/s", "seconds": dt, "threads": threads,
            "bitexact_vs_gpu": same,
            "single_thread": {"value": (mp - 1) / dt1, "selections": mp - 1, "seconds": dt1,
                              "same_prefix": bool(np.array_equal(si, got_i[:mp]))},
            "note": "index build + sampling, host memory, synchronous"}


def cpu_vox_sweep(rf, P, M, fdist, got_i, np):
    """CPU RadiusFPS time per voxel resolution (one thread on a prefix of
    min(M, 4096) selections, the default team on the whole workload)."""
    out = {}
    mp = min(M, 4096)
    for v in (8, 12, 16, 24, 32, 48, 64, 96, 128, 192):
        t0 = time.perf_counter()
        ci, _ = rf.cpu_fps(P, M, 0, n_vox=v, flags=fdist)
        team = time.perf_counter() - t0
        t0 = time.perf_counter()
        si, _ = rf.cpu_fps(P, mp, 0, n_vox=v, flags=fdist, threads=1)
        one = time.perf_counter() - t0
        ok = bool(np.array_equal(ci, got_i) and np.array_equal(si, got_i[:mp]))
        out[str(v)] = {"team_s": team, "one_thread_prefix_s": one, "bitexact": ok}
        log("cpu sweep n_vox %4d: team %.3f s, one thread (%d selections) %.3f s, bitexact %s" % (v, team, mp - 1,
                                                                                               one, ok))
    teams = {}
    for t in (1, 2, 4, 8, 16, 32):
        t0 = time.perf_counter()
        ci, _ = rf.cpu_fps(P, M, 0, flags=fdist, threads=t)
        teams[str(t)] = time.perf_counter() - t0
        log("cpu sweep default bins, %2d threads: %.3f s, bitexact %s" % (t, teams[str(t)],
                                                                          bool(np.array_equal(ci, got_i))))
    out["team_size_s"] = teams
    return out


def run_ablation(rf, idx, M, fdist, got_i, got_d, stream, torch, np):
    """Sampling time of each variant of the paper's ablation on the same index
    (untimed region of the benchmark; the index build is not included)."""
    variants = [
        ("multi_pick", 0),
        ("one_pick", rf.F_SINGLE_PICK),
        ("one_pick_no_skip", rf.F_SINGLE_PICK | rf.F_NO_POINT_SKIP),
        ("one_pick_no_prune", rf.F_NO_PRUNE),
        ("one_pick_no_prune_no_skip", rf.F_NO_PRUNE | rf.F_NO_POINT_SKIP),
        ("unfused", rf.F_UNFUSED),
        ("unfused_no_skip", rf.F_UNFUSED | rf.F_NO_POINT_SKIP),
        ("unfused_no_prune", rf.F_UNFUSED | rf.F_NO_PRUNE),
        ("unfused_no_prune_no_skip", rf.F_UNFUSED | rf.F_NO_PRUNE | rf.F_NO_POINT_SKIP),
    ]
    out = {"note": "sample call only, index reused; one_pick = one persistent kernel with one exchange per "
                   "selection (the paper's fused design); unfused = two launches per selection; "
                   "no_prune = every tile visited; no_skip = no coordinate-wise point skip"}
    for name, fl in variants:
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record(stream)
        oi, od = rf.sample(idx, M, 0, flags=fl | fdist)
        b.record(stream)
        torch.cuda.synchronize()
        ms = a.elapsed_time(b)
        same = bool(np.array_equal(oi.cpu().numpy(), got_i) and
                    np.array_equal(od.cpu().numpy().view(np.uint32), got_d.view(np.uint32)))
        out[name] = {"sample_ms": ms, "bitexact": same}
        log("ablation %-26s %10.2f ms  bitexact %s" % (name, ms, same))
    return out


def cpu_baseline(clouds, ms, gpu_idx, gpu_d2, seconds, euclid=False):
    """The oracle (plain O(N*M) FPS in C, OpenMP over the host cores) on a
    bounded prefix of every cloud's selections, about `seconds` of CPU time in
    all; the prefixes are also checked against the GPU's outputs."""
    import numpy as np
    import oracle
    oracle.build(force=False)
    threads = oracle.num_threads()
    # probe the cost of one selection per point on the first cloud
    mp0 = min(ms[0], 64)
    t0 = time.perf_counter()
    oracle.fps(clouds[0], mp0, 0, threads=0)
    per_pt_sel = (time.perf_counter() - t0) / max(1, (mp0 - 1) * clouds[0].shape[0])
    work = sum(c.shape[0] * (m - 1) for c, m in zip(clouds, ms))
    frac = min(1.0, seconds / max(per_pt_sel * work, 1e-9))
    sel, same = 0, True
    t0 = time.perf_counter()
    for c, m, gi, gd in zip(clouds, ms, gpu_idx, gpu_d2):
        mp = max(2, min(m, int(round(frac * m))))
        ri, rd = oracle.fps(c, mp, 0, threads=0, euclid=euclid)
        sel += mp - 1
        same &= bool(np.array_equal(ri, gi[:mp]) and np.array_equal(rd.view(np.uint32), gd[:mp].view(np.uint32)))
    dt = time.perf_counter() - t0
    total = sum(m for m in ms)
    # context: one host thread, plain FPS and the CPU RadiusFPS of the oracle
    # package on the same prefix of the first cloud (about seconds / 4 each)
    c0, m0 = clouds[0], ms[0]
    mp1 = max(2, min(m0, int(round(min(1.0, 0.25 * seconds / max(per_pt_sel * threads * c0.shape[0] * (m0 - 1),
                                                                     1e-9)) * m0))))
    t1 = time.perf_counter()
    pi, _ = oracle.fps(c0, mp1, 0, threads=1, euclid=euclid)
    t_plain1 = time.perf_counter() - t1
    from paper_2606_06255_amd import default_n_vox
    t1 = time.perf_counter()
    ci, _, _ = oracle.rfps_cpu(c0, mp1, 0, n_vox=default_n_vox(c0.shape[0]))
    t_rfps1 = time.perf_counter() - t1
    single = {"plain_fps_value": (mp1 - 1) / t_plain1, "radiusfps_value": (mp1 - 1) / t_rfps1,
              "radiusfps_speedup": t_plain1 / t_rfps1, "selections": mp1 - 1,
              "same_selections": bool(np.array_equal(pi, gpu_idx[0][:mp1]) and (euclid or np.array_equal(pi, ci)))}
    return {"value": sel / dt, "unit": "selected pts/s", "cores": threads, "kind": "oracle",
            "sample": "first %.1f%% of the selections of every cloud of the same workload (%d of %d selections, "
                      "%d cloud%s), plain O(N*M) FPS in C, OpenMP" % (100 * frac, sel, total - len(ms), len(ms),
                                                                      "s" if len(ms) > 1 else ""),
            "seconds": dt, "bitexact_prefix": same, "single_thread": single}


def run_stages(args, rf, dev, stream):
    """The multi-stage LiDAR workload: one step is all three stages, each an
    index build and FPS of the previous stage's picks (gathered on the device
    by rfps_gather_xyz), as a point backbone down-samples."""
    import numpy as np
    import torch
    import synth

    P = synth.lidar(0)
    sizes = [int(v) for v in synth.lidar_stage_sizes(P.shape[0])]
    ms = sizes[1:]
    K = len(ms)
    xs = [torch.from_numpy(P).to(dev)] + [torch.empty((mm, 3), dtype=torch.float32, device=dev) for mm in ms[:-1]]
    outs = [(torch.empty(mm, dtype=torch.int32, device=dev), torch.empty(mm, dtype=torch.float32, device=dev))
            for mm in ms]
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731
    idxs = [None] * K

    def step(marks=None):
        for k in range(K):
            if marks is not None:
                marks[k][0].record(stream)
            idxs[k] = rf.build_index(xs[k], reuse=idxs[k])
            rf.sample(idxs[k], ms[k], 0, lookahead=args.lookahead, out_idx=outs[k][0], out_d2=outs[k][1])
            if k + 1 < K:
                rf.gather_xyz(xs[k], outs[k][0], out=xs[k + 1])
            if marks is not None:
                marks[k][1].record(stream)

    # ---- timed region ---------------------------------------------------------
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    for k in range(K):
        st = rf.read_status(idxs[k])
        if st != 0:
            raise rf.RfpsError(st, "device status, stage %d" % (k + 1))
    a, b = ev(), ev()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    a.record(stream)
    for _ in range(args.steps):
        step()
    b.record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    ms_per_step = a.elapsed_time(b) / args.steps
    for k in range(K):
        st = rf.read_status(idxs[k])
        if st != 0:
            raise rf.RfpsError(st, "device status, stage %d" % (k + 1))
    got = [(o[0].cpu().numpy().copy(), o[1].cpu().numpy().copy()) for o in outs]
    log("timed %d steps: %.3f ms/step (wall %.3f ms/step)" % (args.steps, ms_per_step,
                                                              1e3 * (wall1 - wall0) / args.steps))
    # ---- untimed: per-stage times and comparators -----------------------------
    marks = [(ev(), ev()) for _ in range(K)]
    step(marks)
    torch.cuda.synchronize()
    stage_ms = [m0.elapsed_time(m1) for m0, m1 in marks]
    pws = rf.PlainWorkspace(P.shape[0], dev)
    plain = [(torch.empty(mm, dtype=torch.int32, device=dev), torch.empty(mm, dtype=torch.float32, device=dev))
             for mm in ms]
    pxs = [xs[0]] + [torch.empty((mm, 3), dtype=torch.float32, device=dev) for mm in ms[:-1]]

    def plain_chain():
        for k in range(K):
            rf.fps_plain(pxs[k], ms[k], 0, variant=0, ws=pws, out_idx=plain[k][0], out_d2=plain[k][1], check=False)
            if k + 1 < K:
                rf.gather_xyz(pxs[k], plain[k][0], out=pxs[k + 1])

    plain_chain()
    torch.cuda.synchronize()
    a, b = ev(), ev()
    a.record(stream)
    plain_chain()
    b.record(stream)
    torch.cuda.synchronize()
    plain_ms = a.elapsed_time(b)
    same = all(np.array_equal(plain[k][0].cpu().numpy(), got[k][0]) and
               np.array_equal(plain[k][1].cpu().numpy().view(np.uint32), got[k][1].view(np.uint32)) for k in range(K))
    total_sel = sum(ms)
    result = {
        "metric": METRIC,
        "value": total_sel / (ms_per_step / 1e3),
        "unit": "selected pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "lidar_stages", "description": WORKLOADS["lidar_stages"], "sizes": sizes,
                   "start": 0, "n_vox": "default per stage", "lookahead": args.lookahead or 2},
        "ms_per_cloud": ms_per_step,
        "stage_ms": stage_ms,
        "comparators": {"plain_persistent_chain_ms": plain_ms},
        "speedup_vs_plain_persistent": plain_ms / ms_per_step,
        "bitexact_vs_plain": bool(same),
    }
    if not args.no_cpu_baseline:
        clouds, cur = [], P
        for k in range(K):
            clouds.append(cur)
            cur = cur[got[k][0]]
        result["cpu_baseline"] = cpu_baseline(clouds, ms, [g[0] for g in got], [g[1] for g in got],
                                              args.cpu_seconds)
    return result


def run_batch(args, rf, dev, stream):
    """The batched workload: 32 uneven clouds, one call per step."""
    import numpy as np
    import torch
    import synth

    xyz, offsets, m = synth.batch(0, b=32)
    B, N, MT = len(m), xyz.shape[0], int(m.sum())
    sizes = np.diff(offsets)
    x = torch.from_numpy(xyz).to(dev)
    off_d = torch.from_numpy(offsets).to(dev)
    m_d = torch.from_numpy(m).to(dev)
    ws = rf.BatchWorkspace(N, B, dev)
    out_i = torch.empty(MT, dtype=torch.int32, device=dev)
    out_d = torch.empty(MT, dtype=torch.float32, device=dev)
    ev = lambda: torch.cuda.Event(enable_timing=True)  # noqa: E731

    # parameters from the autotuner (untimed; part of the warm-up)
    t0 = time.perf_counter()
    chosen, tuned_ms, _ = rf.autotune_batched(x, offsets, m, reps=3, ws=ws)
    tune_s = time.perf_counter() - t0
    log("autotuner: %s, %.2f ms per batch (%.1f s)" % (chosen, tuned_ms, tune_s))
    kw = dict(groups=chosen["groups"], lookahead=chosen["lookahead"], tile=chosen["tile"])

    def call(flags=0, **over):
        p = dict(kw)
        p.update(over)
        rf.sample_batched(x, off_d, m_d, m_total=MT, ws=ws, out_idx=out_i, out_d2=out_d, check=False,
                          flags=flags, **p)

    side = torch.cuda.Stream(dev)
    side.wait_stream(stream)
    with torch.cuda.stream(side):
        call()
    stream.wait_stream(side)
    torch.cuda.synchronize()
    graph = torch.cuda.CUDAGraph()
    with torch.cuda.graph(graph):
        call()

    # ---- timed region: graph replays ----------------------------------------
    for _ in range(args.warmup):
        graph.replay()
    torch.cuda.synchronize()
    st = rf.batched_read_status(ws)
    if st != 0:
        raise rf.RfpsError(st, "device status")
    a, b = ev(), ev()
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    a.record(stream)
    for _ in range(args.steps):
        graph.replay()
    b.record(stream)
    torch.cuda.synchronize()
    wall1 = time.perf_counter()
    ms_per_step = a.elapsed_time(b) / args.steps
    st = rf.batched_read_status(ws)
    if st != 0:
        raise rf.RfpsError(st, "device status")
    got_i = out_i.cpu().numpy().copy()
    got_d = out_d.cpu().numpy().copy()
    log("timed %d graph replays: %.3f ms/batch (wall %.3f ms)" % (args.steps, ms_per_step,
                                                                  1e3 * (wall1 - wall0) / args.steps))

    def timed(fn, reps):
        fn()
        torch.cuda.synchronize()
        a, b = ev(), ev()
        a.record(stream)
        for _ in range(reps):
            fn()
        b.record(stream)
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    reps = max(1, min(args.steps, 5))
    eager_ms = timed(call, reps)
    default_ms = timed(lambda: call(groups=0, lookahead=0, tile=0), reps)
    same_default = np.array_equal(out_i.cpu().numpy(), got_i)

    # telemetry of the tuned call (roofline of the whole call)
    call(flags=rf.F_TELEMETRY)
    tel = rf.batched_read_telemetry(ws)
    NT = tel["tiles"]
    # as for one cloud, with the sphere tests counted by the sampler (every
    # tile of a cloud against every selection of that cloud)
    alg_bytes = (16 * N + 20 * NT + 24 * tel["tile_tests"] + 16 * tel["points_visited"]
                 + 4 * tel["points_updated"] + 12 * tel["tiles_resynced"] + 8 * (MT - B))
    achieved = alg_bytes / (ms_per_step / 1e3) / 1e9
    visit = tel["points_visited"] / max(1, int((sizes.astype(np.int64) * (m.astype(np.int64) - 1)).sum()))

    # ---- comparators: per-cloud launches of the single-cloud path -------------
    comps = {}
    o = np.concatenate([[0], np.cumsum(m)])
    per_i = torch.empty(MT, dtype=torch.int32, device=dev)
    per_d = torch.empty(MT, dtype=torch.float32, device=dev)
    order = np.argsort(-sizes, kind="stable")
    idx = rf.build_index(x[offsets[order[0]]:offsets[order[0] + 1]])

    def per_cloud():
        nonlocal idx
        for c in range(B):
            idx = rf.build_index(x[offsets[c]:offsets[c + 1]], reuse=idx)
            rf.sample(idx, int(m[c]), 0, out_idx=per_i[o[c]:o[c + 1]], out_d2=per_d[o[c]:o[c + 1]])

    comps["per_cloud_rfps_ms"] = timed(per_cloud, 2)
    same_per = np.array_equal(per_i.cpu().numpy(), got_i) and np.array_equal(
        per_d.cpu().numpy().view(np.uint32), got_d.view(np.uint32))
    pws = rf.PlainWorkspace(int(sizes.max()), dev)

    def per_cloud_plain():
        for c in range(B):
            rf.fps_plain(x[offsets[c]:offsets[c + 1]], int(m[c]), 0, variant=0, ws=pws,
                         out_idx=per_i[o[c]:o[c + 1]], out_d2=per_d[o[c]:o[c + 1]], check=False)

    comps["per_cloud_plain_persistent_ms"] = timed(per_cloud_plain, 1)
    same_plain = np.array_equal(per_i.cpu().numpy(), got_i)
    comps["batched_eager_tuned_ms"] = eager_ms
    comps["batched_eager_default_ms"] = default_ms

    result = {
        "metric": METRIC,
        "value": MT / (ms_per_step / 1e3),
        "unit": "selected pts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": "batch", "description": WORKLOADS["batch"], "clouds": B, "n_points": N,
                   "m_total": MT, "n_min": int(sizes.min()), "n_max": int(sizes.max()), "start": 0,
                   "n_vox": "per-cloud default", "tuned": chosen, "launch": "hipGraph replay"},
        "ms_per_cloud": ms_per_step / B,
        "autotune": {"chosen": chosen, "median_ms": tuned_ms, "seconds": tune_s},
        "pruning": {"point_visit_fraction": visit, **tel},
        # as for one cloud: every team waits on one XCD-local exchange per
        # round, so the call is latency-bound; the byte fractions stand beside
        # it (no bare-exchange floor is measured for teams)
        "roofline": {"bound": "latency", "kernel": "whole batched call (index build + k_rfps_rounds_batched)",
                     "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": None, "fractions": {"hbm_algorithmic": achieved / HBM_PEAK_GBS,
                                                    "lds": achieved / LDS_PEAK_GBS},
                     "lds_peak_gbs": LDS_PEAK_GBS, "exchange_rounds": tel["exchanges"],
                     "alg_bytes_per_launch": alg_bytes},
        "comparators": comps,
        "speedup_vs_per_cloud_rfps": comps["per_cloud_rfps_ms"] / ms_per_step,
        "speedup_vs_per_cloud_plain_persistent": comps["per_cloud_plain_persistent_ms"] / ms_per_step,
        "graph_vs_eager": eager_ms / ms_per_step,
        "bitexact_vs_per_cloud": bool(same_per and same_plain and same_default),
    }
    if not args.no_cpu_baseline:
        clouds = [xyz[offsets[c]:offsets[c + 1]] for c in range(B)]
        result["cpu_baseline"] = cpu_baseline(clouds, [int(v) for v in m], [got_i[o[c]:o[c + 1]] for c in range(B)],
                                              [got_d[o[c]:o[c + 1]] for c in range(B)], args.cpu_seconds)
    return result


if __name__ == "__main__":
    sys.exit(main())
