"""Benchmark of the voting transform on one MI355X.

A step is one pass of the hot path over one chip's catalog, already resident
in HBM: sas_vote (reference epoch, window index, dense LDS vote over the
whole velocity grid) followed by sas_peaks (device -> host candidates in
canonical order).  Default workload: the wide-field chip (2048x4096 px,
100 epochs over 4 h, 3000 noise detections per epoch plus 200 movers, 4 px
bins, sector grid of 84,351 velocities, N_min = 25).

--workload night runs the batched night instead: 64 chips (seeded wide or
fast style, 5e4-5e5 detections, 40-120 epochs, each with its own grid and
threshold) voted by one batched launch per kernel class, with launch shapes
chosen by the autotuner per chip style.

Prints one JSON line (rank 0).  --gpus above 1 is refused: the benchmark
measures one GPU.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# MI355X published / derived peaks
HBM_PEAK_GBS = 8000.0
N_CU, CLOCK_GHZ = 256, 2.4
SIMD_PER_CU, LANES_PER_SIMD = 4, 16
# 32-bit integer vector ops: one per lane per clock on 4 x 16-lane SIMDs per
# CU (the published 157.3 TFLOP/s fp32 vector peak counts an FMA as 2 and
# packed fp32 as 2 more)
INT_PEAK_TOPS = N_CU * SIMD_PER_CU * LANES_PER_SIMD * CLOCK_GHZ / 1000.0
# Packed 16-bit integer ops (v_pk_sub_u16, v_pk_lshrrev_b16, v_dot2_u32_u16):
# two halves per lane per clock.  Votes of a packed plan run at this rate.
INT16X2_PEAK_TOPS = 2 * INT_PEAK_TOPS
# LDS: one 4-byte access per bank per clock, 32 banks per CU; an atomic add
# reads and writes its word, so a 64-lane ds_add_u32 without bank conflicts
# takes 4 clocks: 16 lane-atomics per CU per clock
LDS_BANKS = 32
LDS_ATOMIC_PEAK = N_CU * (LDS_BANKS // 2) * CLOCK_GHZ * 1e9  # lane atomics per second
# Integer operations of one vote on the dense path: x - S_x, y - S_y, the two
# floor divisions by the cell width (shifts), and the histogram word index
# (bin row * row pitch + bin column * lanes + lane: one multiply-add and one
# shift-add).  The count increment itself is the LDS atomic.
OPS_PER_VOTE = 6
# A weighted vote also takes its weight out of the staged entry (one and).
OPS_PER_WEIGHTED_VOTE = 7
VOTE_KERNEL = "k_vote_dense"


def _night(n_chips, tune, log, full_tune=False):
    """The batched night: chips with their own plans, thresholds and
    autotuned launch shapes (one tuning per shape class: bin width, lattice
    spacing, grid shape, and epoch and detection counts by powers of two)."""
    import torch

    from paper_2509_26279_amd import autotune, sas, synth
    chips, tuned = [], {}
    for p in synth.night_chip_params(4, n_chips):
        wl = synth.make_night_chip(p, 0)
        v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
        n_min = wl.n_min
        if p["style"] == "fast":  # threshold rule of Sec. 2.2 for this chip
            area = float(wl.width_px * wl.height_px)
            mu = wl.n / wl.n_epochs * wl.bin_px ** 2 / area
            n_min = sas.threshold_n_min(wl.n_epochs, mu, len(v) * area / wl.bin_px ** 2)
        x = torch.as_tensor(wl.x_q8).cuda()
        y = torch.as_tensor(wl.y_q8).cuda()
        e = torch.as_tensor(wl.epoch).cuda()
        key = autotune.shape_class(wl.binw_q8, sas.grid_spacing(wl.binw_q8, wl.span_q16),
                                   wl.n_epochs, wl.n, wl.grid.shape)
        if tune and key not in tuned:
            log("tuning class %s on chip %d" % (key, p["chip"]))
            cands = (autotune.candidates({"n_det_hint": wl.n}) if full_tune else
                     [{}, {"groups": 1}, {"groups": 2}, {"groups": 4}])
            r = autotune.tune(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8, x, y, e,
                              cands=cands, log=log)
            tuned[key] = {k: v_ for k, v_ in r["tuning"].items() if k != "n_det_hint"}
        tun = dict(tuned.get(key, {}), n_det_hint=wl.n)
        plan = sas.Plan(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8, tuning=tun)
        chips.append({"wl": wl, "v": v, "plan": plan, "x": x, "y": y, "e": e, "n_min": n_min,
                      "style": p["style"]})
    return chips, tuned


def run_night(args):
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas
    log = lambda m: print(m, file=sys.stderr, flush=True)
    chips, tuned = _night(args.chips, not args.no_tune, log, args.full_tune)
    b = sas.Batch([(c["plan"], c["x"], c["y"], c["e"]) for c in chips], cand_cap=1 << 21)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        b.vote()
        for k in range(len(chips)):
            b.peaks(k)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, z in evs:
        a.record(stream)
        z.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_cand = 0
    for k in range(args.steps):
        b.set_probe(evs[k][0], evs[k][1])
        b.vote()
        n_cand = sum(len(b.peaks(c)) for c in range(len(chips)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    b.set_probe(None, None)
    kernel_ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    ms_step = wall * 1000.0 / args.steps
    votes = float(sum(c["wl"].n * len(c["v"]) for c in chips))
    achieved = OPS_PER_VOTE * votes / (kernel_ms * 1e-3) / 1e12
    # the peak of the night's vote mix: each chip's votes at its plan's rate
    peak = votes / sum(c["wl"].n * len(c["v"]) /
                       (INT16X2_PEAK_TOPS if c["plan"].info()["packed"] else INT_PEAK_TOPS)
                       for c in chips)
    n_fast = sum(c["style"] == "fast" for c in chips)
    rec = {
        "metric": "detection-velocity votes/s per chip", "value": votes / (ms_step * 1e-3),
        "unit": "votes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "night: %d chips (%d wide-style, %d fast-style), detections "
                               "log-uniform 5e4-5e5, 40-120 epochs, one batched launch"
                               % (len(chips), len(chips) - n_fast, n_fast),
                   "n_detections": int(sum(c["wl"].n for c in chips)),
                   "votes": votes, "parallelism": "single-gpu"},
        "candidates_per_s": n_cand / (ms_step * 1e-3), "n_candidates": n_cand,
        "vote_kernels_ms": kernel_ms, "tuned": tuned,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "Tops/s", "frac": achieved / peak, "traffic": None,
                     "kernel": "k_vote_dense_batch", "ops_per_vote": OPS_PER_VOTE},
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(chips[0]["wl"], chips[0]["v"], args.cpu_seconds,
                                           chips[0]["n_min"])
    b.close()
    for c in chips:
        c["plan"].close()
    print(json.dumps(rec), flush=True)


def _workload(name):
    from paper_2509_26279_amd import synth
    if name == "wide":
        return synth.make_wide()
    if name == "fast":
        return synth.make_fast()
    if name == "tiny":
        return synth.make_tiny()
    raise SystemExit("unknown workload " + name)


def _kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_2509_26279_amd", "csrc", "vote_dense.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload):
    """HBM bytes per vote-kernel launch from the committed PMC summary, or
    None when there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (VOTE_KERNEL, workload))
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(wl, v, seconds, n_min=None):
    """The oracle as it stands, on the host cores, over a seeded velocity sample."""
    import numpy as np

    import oracle
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    rng = np.random.default_rng(0)
    probe = np.sort(rng.choice(len(v), size=min(threads, len(v)), replace=False))
    t0 = time.perf_counter()
    n_min = wl.n_min if n_min is None else n_min
    oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[probe], wl.binw_q8, n_min,
                "epochs", 255, threads=threads)
    dt = time.perf_counter() - t0
    k = int(max(threads, min(len(v), threads * round(seconds / max(dt, 1e-3)))))
    sample = np.sort(rng.choice(len(v), size=k, replace=False))
    t0 = time.perf_counter()
    c = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[sample], wl.binw_q8, n_min,
                    "epochs", 255, threads=threads)
    dt = time.perf_counter() - t0
    return {"value": wl.n * k / dt, "unit": "votes/s", "cores": threads, "kind": "oracle",
            "sample": "%d of %d velocities (seeded), full catalog of %d detections, %.1f s"
                      % (k, len(v), wl.n, dt),
            "candidates": int(len(c))}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="wide")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chips", type=int, default=64, help="night workload: number of chips")
    ap.add_argument("--no-tune", action="store_true", help="night workload: planner defaults")
    ap.add_argument("--full-tune", action="store_true",
                    help="night workload: the autotuner's whole candidate list per chip style")
    ap.add_argument("--extract", action="store_true",
                    help="also time the greedy cluster extraction over the step's candidates")
    ap.add_argument("--extract-rounds", type=int, default=0,
                    help="parallel rounds of the extraction (0 default, -1 one take at a time)")
    ap.add_argument("--refine", action="store_true",
                    help="also time Steps 4-6 (FAST-MCD refine, gather, iterate) over the "
                         "clusters of the greedy extraction (implies --extract)")
    ap.add_argument("--refine-starts", type=int, default=500,
                    help="random starts of FAST-MCD per fit (at most 1024)")
    ap.add_argument("--weighted", choices=["epochs", "detections"], default=None,
                    help="also time the weighted vote of the same catalog (likelihood weights "
                         "of the detections' SNR, threshold N_min x the mean weight)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)

    if args.workload == "night":
        run_night(args)
        return

    import numpy as np
    import torch

    from paper_2509_26279_amd import sas

    wl = _workload(args.workload)
    v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    count_sat = 255 if wl.count_dtype == "u8" else 65535
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, count_sat=count_sat,
                    tuning={"n_det_hint": wl.n})
    info = plan.info()
    s = sas.Search(plan, wl.n, cand_cap=1 << 22)
    x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
    stream = torch.cuda.current_stream()

    for _ in range(args.warmup):
        s.vote(x, y, e)
        out = s.peaks()
    torch.cuda.synchronize()

    # events around the whole step (vote + peaks) and, through the plan's
    # probe, around the vote kernel alone on the stream it is launched on
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:  # create the underlying HIP events
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.set_probe(evs[k][0], evs[k][1])
        s.vote(x, y, e)
        out = s.peaks()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_probe(None, None)
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ms_step = wall * 1000.0 / args.steps
    votes = float(wl.n) * len(v)
    n_cand = len(out)

    achieved = OPS_PER_VOTE * votes / (kernel_ms * 1e-3) / 1e12
    peak = INT16X2_PEAK_TOPS if info.get("packed") else INT_PEAK_TOPS
    rec = {
        "metric": "detection-velocity votes/s per chip",
        "value": votes / (ms_step * 1e-3),
        "unit": "votes/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": "%s chip: %dx%d px, %d epochs over %.0f h, %d detections, "
                               "%d velocities, %.0f px bins, N_min %d"
                               % (wl.name, wl.width_px, wl.height_px, wl.n_epochs, wl.span_h,
                                  wl.n, len(v), wl.bin_px, wl.n_min),
                   "n_detections": wl.n, "n_velocities": int(len(v)),
                   "n_epochs": wl.n_epochs, "parallelism": "single-gpu"},
        "candidates_per_s": n_cand / (ms_step * 1e-3),
        "n_candidates": n_cand,
        "vote_kernel_ms": kernel_ms,
        "vote_kernel_votes_per_s": votes / (kernel_ms * 1e-3),
        "plan": info,
        "roofline": {"bound": "alu", "achieved": achieved, "peak": peak,
                     "unit": "Tops/s", "frac": achieved / peak,
                     "traffic": _traffic(wl.name), "kernel": VOTE_KERNEL,
                     "ops_per_vote": OPS_PER_VOTE,
                     "ops": "int16x2 packed" if info.get("packed") else "int32",
                     "lds_atomic_frac": votes / (kernel_ms * 1e-3) / LDS_ATOMIC_PEAK},
    }
    if args.extract or args.refine:
        # Step 3's greedy extraction over the candidates of the last vote
        # (not part of the step above): wall time of the whole call
        ext = []
        for k in range(args.warmup + args.steps):
            s.vote(x, y, e)
            s.peaks()
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            clusters, _ = s.extract(wl.n, rounds=args.extract_rounds)
            if k >= args.warmup:
                ext.append((time.perf_counter() - t1) * 1000.0)
        rec["extract"] = {"ms": float(np.mean(ext)), "n_clusters": int(len(clusters)),
                          "n_cells": n_cand, "rounds": args.extract_rounds}
        if args.refine:
            from paper_2509_26279_amd import synth
            _, owner = s.extract(wl.n)
            order = np.argsort(owner, kind="stable")
            own = owner[order]
            groups = [order[own == k] for k in range(len(clusters))]
            starts = synth.mcd_starts(7, args.refine_starts)
            ref = []
            for k in range(args.warmup + args.steps):
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                recs, _, _ = s.refine(x, y, e, groups, starts, subsets=False)
                if k >= args.warmup:
                    ref.append((time.perf_counter() - t1) * 1000.0)
            st = {sas.REFINE_STATUS[int(c)]: int((recs["status"] == c).sum())
                  for c in np.unique(recs["status"])}
            rec["refine"] = {"ms": float(np.mean(ref)), "n_clusters": len(groups),
                             "points": int(sum(len(g) for g in groups)),
                             "rounds_mean": float(recs["rounds"].mean()) if len(recs) else 0.0,
                             "status": st, "starts": args.refine_starts}
    if args.weighted:
        rec["weighted"] = time_weighted(args, wl, v, count_sat)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(wl, v, args.cpu_seconds)
    plan.close()
    print(json.dumps(rec), flush=True)


def time_weighted(args, wl, v, count_sat):
    """The step of main() with a weighted plan (not the headline value)."""
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas, synth
    w = synth.likelihood_weights(wl.snr)
    n_min = int(round(wl.n_min * float(w.mean())))
    mode = "weighted_" + args.weighted
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, n_min, wl.extent_q8, mode=mode,
                    count_sat=65535, tuning={"n_det_hint": wl.n,
                                             "weight_hint": int(round(float(w.mean())))})
    info = plan.info()
    s = sas.Search(plan, wl.n, cand_cap=1 << 22)
    x, y, e, wd = s.upload(wl.x_q8, wl.y_q8, wl.epoch, w)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        s.vote(x, y, e, wd)
        s.peaks()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
        a.record(stream)
        b.record(stream)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        plan.set_probe(evs[k][0], evs[k][1])
        s.vote(x, y, e, wd)
        out = s.peaks()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    plan.set_probe(None, None)
    kernel_ms = float(np.mean([a.elapsed_time(b) for a, b in evs]))
    ms_step = wall * 1000.0 / args.steps
    votes = float(wl.n) * len(v)
    achieved = OPS_PER_WEIGHTED_VOTE * votes / (kernel_ms * 1e-3) / 1e12
    plan.close()
    return {"mode": mode, "n_min": n_min, "weights": "round(2 snr^2), capped at 255",
            "value": votes / (ms_step * 1e-3), "unit": "votes/s", "ms_per_step": ms_step,
            "vote_kernel_ms": kernel_ms, "n_candidates": int(len(out)), "plan": info,
            "roofline": {"bound": "alu", "achieved": achieved, "peak": INT_PEAK_TOPS,
                         "unit": "Tops/s", "frac": achieved / INT_PEAK_TOPS,
                         "kernel": VOTE_KERNEL, "ops_per_vote": OPS_PER_WEIGHTED_VOTE,
                         "ops": "int32"}}


if __name__ == "__main__":
    main()
