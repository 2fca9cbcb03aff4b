"""Benchmark of the voting transform on one MI355X.

A step is one pass of the hot path over the workload's catalogs, already
resident in HBM: the vote (reference epoch, window index, dense LDS vote over
the whole velocity grid of every chip, refinement of flagged cells) followed
by sas_peaks of every chip (device -> host candidates in canonical order).

Default workload: the batched night, the largest single-GPU configuration:
64 chips (seeded wide or fast style, 5e4-5e5 detections, 40-120 epochs, each
with its own velocity grid and threshold) voted by one persistent launch per
kernel class, captured once as a HIP graph and replayed every step; launch
shapes come from the committed tuning cache (no tuning in the timed run).
--workload wide|fast|tiny runs one chip's sas_vote + sas_peaks instead.

Prints one JSON line.  --gpus above 1 is refused: the benchmark measures one
GPU.  --ceilings prints the measured unit rates instead (LDS atomics, integer
VALU, HBM copy).
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
# Packed 16-bit integer ops: two halves per lane per clock.
INT16X2_PEAK_TOPS = 2 * INT_PEAK_TOPS
# LDS: one 4-byte access per bank per clock, 32 banks per CU; an atomic add
# reads and writes its word, so a 64-lane ds_add_u32 without bank conflicts
# takes 4 clocks: 16 lane-atomics per CU per clock.  Each vote is one lane
# of one LDS atomic instruction.
LDS_BANKS = 32
LDS_ATOMIC_PEAK = N_CU * (LDS_BANKS // 2) * CLOCK_GHZ * 1e9  # lane atomics per second
# Integer operations of one vote on the dense path: x - S_x, y - S_y, the two
# floor divisions by the cell width (shifts), and the histogram word index
# (one multiply-add and one shift-add).  The count increment is the atomic.
OPS_PER_VOTE = 6
OPS_PER_WEIGHTED_VOTE = 7
VOTE_KERNEL = "k_vote_dense"
BATCH_KERNEL = "k_vote_dense_batch"


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _lds_roofline(kernel, instr, kernel_s, votes, alu_peak_tops, traffic):
    """Roofline of a vote kernel against the LDS atomic unit: `instr`
    64-lane atomic vote instructions (device counter) over the kernel time.
    The algorithmic rate (N |V| votes over the same time) is reported next
    to it: coverage pruning skips tiles that cannot hold a candidate, so the
    kernel issues fewer lane atomics than N |V|."""
    lanes = 64.0 * instr
    achieved = lanes / kernel_s
    return {"bound": "lds_atomic", "achieved": achieved, "peak": LDS_ATOMIC_PEAK,
            "unit": "lane-atomics/s", "frac": achieved / LDS_ATOMIC_PEAK, "traffic": traffic,
            "kernel": kernel, "lane_atomics_per_launch": lanes,
            "algorithmic_votes_per_launch": votes,
            "algorithmic_votes_per_s": votes / kernel_s,
            "algorithmic_frac": votes / kernel_s / LDS_ATOMIC_PEAK,
            "alu_frac": OPS_PER_VOTE * lanes / kernel_s / (alu_peak_tops * 1e12),
            "ops_per_vote": OPS_PER_VOTE}


# --------------------------------------------------------------------------- night

def run_night(args):
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas
    t_setup = time.perf_counter()
    from paper_2509_26279_amd import night
    chips, tuned, missing = night.setup(args.chips, args.cache, args.retune, args.tune_set, log)
    b = sas.Batch([(c["plan"], c["x"], c["y"], c["e"]) for c in chips], cand_cap=1 << 21)
    stream = torch.cuda.current_stream()
    for _ in range(max(args.warmup, 1)):
        b.vote()
        eager = [b.peaks(k) for k in range(len(chips))]
    torch.cuda.synchronize()
    graph = None
    if not args.no_graph:  # one capture of the whole batch, replayed per step
        graph = torch.cuda.CUDAGraph()
        with torch.cuda.graph(graph):
            b.vote(stream=torch.cuda.current_stream())
        graph.replay()
        for k in range(len(chips)):
            if not np.array_equal(b.peaks(k), eager[k]):
                raise RuntimeError("graph replay of chip %d differs from the eager vote" % k)
    setup_s = time.perf_counter() - t_setup
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    n_cand = 0
    for _ in range(args.steps):
        if graph is not None:
            graph.replay()
        else:
            b.vote()
        n_cand = sum(len(b.peaks(k)) for k in range(len(chips)))
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms_step = wall * 1000.0 / args.steps
    # the vote kernels alone, on the launch stream, eager, after the timed
    # region: events around them, then one more vote with the LDS atomic
    # counter on (counting adds work, so it is not timed)
    reps = 2
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(reps)]
    for a, z in evs:
        a.record(stream)
        z.record(stream)
    torch.cuda.synchronize()
    for a, z in evs:
        b.set_probe(a, z)
        b.vote()
    torch.cuda.synchronize()
    b.set_probe(None, None)
    kernel_ms = float(np.mean([a.elapsed_time(z) for a, z in evs]))
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    b.set_counter(counter)
    b.vote()
    torch.cuda.synchronize()
    b.set_counter(None)
    instr = float(counter.item())
    votes = float(sum(c["wl"].n * len(c["v"]) for c in chips))
    # the ALU peak of the night's vote mix: each chip's votes at its plan's rate
    alu_peak = votes / sum(c["wl"].n * len(c["v"]) /
                           (INT16X2_PEAK_TOPS if c["plan"].info()["packed"] else INT_PEAK_TOPS)
                           for c in chips)
    infos = [c["plan"].info() for c in chips]
    n_fast = sum(c["style"] == "fast" for c in chips)
    rec = {
        "metric": "detection-velocity votes/s per chip", "value": votes / (ms_step * 1e-3),
        "unit": "votes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "night: %d chips (%d wide-style, %d fast-style), detections "
                               "log-uniform 5e4-5e5, 40-120 epochs, one batched launch per "
                               "kernel class, replayed as a captured graph"
                               % (len(chips), len(chips) - n_fast, n_fast),
                   "n_chips": len(chips),
                   "n_detections": int(sum(c["wl"].n for c in chips)),
                   "n_velocities": int(sum(len(c["v"]) for c in chips)),
                   "votes": votes, "parallelism": "single-gpu"},
        "per_ccd_chip": {"ms": ms_step / len(chips), "chips_per_s": len(chips) / (wall /
                                                                                    args.steps),
                         "votes_per_s_mean_chip": votes / len(chips) / (ms_step * 1e-3)},
        "candidates_per_s": n_cand / (ms_step * 1e-3), "n_candidates": n_cand,
        "vote_kernels_ms": kernel_ms, "graph": graph is not None,
        "tiles": int(sum(i["n_tiles"] for i in infos)),
        "tiles_voted": int(sum(i["n_tiles_kept"] for i in infos)),
        "tuning_cache": os.path.relpath(args.cache, ROOT), "tuned_classes": len(tuned),
        "untuned_classes": missing, "setup_s": setup_s,
        "roofline": _lds_roofline(BATCH_KERNEL, instr, kernel_ms * 1e-3, votes, alu_peak,
                                  _traffic("night", BATCH_KERNEL)),
    }
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline_night(chips, args.cpu_seconds)
    b.close()
    for c in chips:
        c["plan"].close()
    print(json.dumps(rec), flush=True)


# --------------------------------------------------------------------------- one chip

def _workload(name):
    from paper_2509_26279_amd import synth
    makers = {"wide": synth.make_wide, "fast": synth.make_fast, "tiny": synth.make_tiny}
    if name not in makers:
        raise SystemExit("unknown workload " + name)
    return makers[name]()


def _kernel_source_hash():
    import hashlib
    src = os.path.join(ROOT, "paper_2509_26279_amd", "csrc", "vote_dense.hip")
    with open(src, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def _traffic(workload, kernel=VOTE_KERNEL):
    """HBM bytes per vote-kernel launch from the committed PMC summary, or
    None when there is none or the kernel source changed since."""
    path = os.path.join(ROOT, "profiles", "traffic_%s_%s.json" % (kernel, workload))
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha256_16") != _kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def run_chip(args):
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas
    from paper_2509_26279_amd import autotune
    wl = _workload(args.workload)
    v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    count_sat = 255 if wl.count_dtype == "u8" else 65535
    # launch shape of the chip's shape class from the tuning cache (the
    # planner's own choice when the class is not cached; --retune times it)
    key = autotune.shape_class(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, wl.n)
    xt = torch.as_tensor(wl.x_q8).cuda()
    yt = torch.as_tensor(wl.y_q8).cuda()
    et = torch.as_tensor(wl.epoch).cuda()
    tun = None if args.retune else autotune.cached(key, args.cache)
    if tun is None and args.retune:
        cands = [{}, {"groups": 1}, {"groups": 2}, {"groups": 4}] if args.tune_set == "small" \
            else None
        r = autotune.tune(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, xt, yt, et,
                          count_sat=count_sat, base={"n_det_hint": wl.n}, cands=cands, reps=2,
                          log=log)
        tun = {k: v_ for k, v_ in r["tuning"].items() if k != "n_det_hint"}
        autotune.store(key, tun, args.cache)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, count_sat=count_sat,
                    tuning=dict(tun or {}, n_det_hint=wl.n))
    info = plan.info()
    s = sas.Search(plan, wl.n, cand_cap=1 << 22)
    x, y, e = xt, yt, et
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        s.vote(x, y, e)
        out = s.peaks()
    torch.cuda.synchronize()
    # events around the vote kernel alone (the plan's probe, on its launch
    # stream) in every timed step; the LDS atomic counter in one more vote
    # after the timed region (counting adds work, so it is not timed)
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    for a, b in evs:
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
    counter = torch.zeros(1, dtype=torch.int64, device="cuda")
    plan.set_counter(counter)
    s.vote(x, y, e)
    torch.cuda.synchronize()
    plan.set_counter(None)
    instr = float(counter.item())
    ms_step = wall * 1000.0 / args.steps
    votes = float(wl.n) * len(v)
    peak = INT16X2_PEAK_TOPS if info.get("packed") else INT_PEAK_TOPS
    rec = {
        "metric": "detection-velocity votes/s per chip", "value": votes / (ms_step * 1e-3),
        "unit": "votes/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_step, "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "%s chip: %dx%d px, %d epochs over %.0f h, %d detections, "
                               "%d velocities, %.0f px bins, N_min %d"
                               % (wl.name, wl.width_px, wl.height_px, wl.n_epochs, wl.span_h,
                                  wl.n, len(v), wl.bin_px, wl.n_min),
                   "n_detections": wl.n, "n_velocities": int(len(v)),
                   "n_epochs": wl.n_epochs, "parallelism": "single-gpu"},
        "candidates_per_s": len(out) / (ms_step * 1e-3), "n_candidates": len(out),
        "vote_kernel_ms": kernel_ms, "vote_kernel_votes_per_s": votes / (kernel_ms * 1e-3),
        "plan": info, "tuning_class": key, "tuning": tun or {},
        "tuning_cache": os.path.relpath(args.cache, ROOT),
        "roofline": _lds_roofline(VOTE_KERNEL, instr, kernel_ms * 1e-3, votes, peak,
                                  _traffic(wl.name)),
    }
    if args.extract or args.refine:
        rec.update(time_extract_refine(args, wl, s, x, y, e, len(out)))
    if args.weighted:
        rec["weighted"] = time_weighted(args, wl, v)
    if args.sort_sample:
        rec["sort_path"] = time_sort_path(args, wl, v, count_sat, x, y, e)
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline([(wl, v, wl.n_min)], args.cpu_seconds)
    plan.close()
    print(json.dumps(rec), flush=True)


def time_extract_refine(args, wl, s, x, y, e, n_cand):
    """Step 3's greedy extraction (and Steps 4-6) over the candidates of the
    last vote: wall time of the whole call (not part of the step above)."""
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas, synth
    out = {}
    ext = []
    for k in range(args.warmup + args.steps):
        s.vote(x, y, e)
        s.peaks()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        clusters, _ = s.extract(wl.n, rounds=args.extract_rounds)
        if k >= args.warmup:
            ext.append((time.perf_counter() - t1) * 1000.0)
    out["extract"] = {"ms": float(np.mean(ext)), "n_clusters": int(len(clusters)),
                      "n_cells": n_cand, "rounds": args.extract_rounds}
    if args.refine:
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
        out["refine"] = {"ms": float(np.mean(ref)), "n_clusters": len(groups),
                         "points": int(sum(len(g) for g in groups)),
                         "rounds_mean": float(recs["rounds"].mean()) if len(recs) else 0.0,
                         "status": st, "starts": args.refine_starts}
    return out


def time_sort_path(args, wl, v, count_sat, x, y, e):
    """The sort-by-bin-key path against the dense path on a seeded block of
    the grid (not the headline value): vote-kernel time of each, identical
    candidate lists required."""
    import numpy as np
    import torch

    from paper_2509_26279_amd import sas
    rng = np.random.default_rng(11)
    k = min(args.sort_sample, len(v))
    start = int(rng.integers(0, len(v) - k + 1))
    vs = v[start:start + k]  # consecutive velocities: one block of the lattice
    out = {"velocities": k, "first_v_idx": start, "n_detections": wl.n}
    lists = {}
    for path in ("sort", "dense"):
        plan = sas.Plan(vs, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8, count_sat=count_sat,
                        path=path, tuning={"n_det_hint": wl.n})
        s = sas.Search(plan, wl.n, cand_cap=1 << 22)
        s.vote(x, y, e)
        lists[path] = s.peaks()
        ts = []
        for _ in range(max(args.steps, 2)):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            b.record()
            torch.cuda.synchronize()
            plan.set_probe(a, b)
            s.vote(x, y, e)
            torch.cuda.synchronize()
            ts.append(a.elapsed_time(b))
        plan.set_probe(None, None)
        info = plan.info()
        plan.close()
        ms = float(np.median(ts))
        out[path] = {"ms": ms, "votes_per_s": wl.n * k / (ms * 1e-3), "blocks": info["n_blocks"]}
    if not np.array_equal(lists["sort"], lists["dense"]):
        raise RuntimeError("sort and dense paths disagree on the sampled block")
    out["n_candidates"] = int(len(lists["dense"]))
    out["dense_over_sort"] = out["sort"]["ms"] / out["dense"]["ms"]
    return out


def time_weighted(args, wl, v):
    """The step of run_chip() with a weighted plan (not the headline value)."""
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


# --------------------------------------------------------------------------- CPU baseline

def _threads():
    threads = len(os.sched_getaffinity(0))
    if os.environ.get("OMP_NUM_THREADS"):
        threads = min(threads, int(os.environ["OMP_NUM_THREADS"]))
    return threads


def cpu_baseline(items, seconds):
    """The oracle as it stands, on the host cores, over seeded velocity
    samples of the given (workload, grid, threshold) items, about `seconds`
    of work in all; votes/s over the whole sample."""
    import numpy as np

    import oracle
    threads = _threads()
    per = seconds / len(items)
    votes, total_s, parts = 0.0, 0.0, []
    for wl, v, n_min in items:
        rng = np.random.default_rng(0)
        probe = np.sort(rng.choice(len(v), size=min(threads, len(v)), replace=False))
        t0 = time.perf_counter()
        oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[probe], wl.binw_q8, n_min,
                    "epochs", 65535, threads=threads)
        dt = time.perf_counter() - t0
        k = int(max(threads, min(len(v), threads * round(per / max(dt, 1e-3)))))
        sample = np.sort(rng.choice(len(v), size=k, replace=False))
        t0 = time.perf_counter()
        oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v[sample], wl.binw_q8, n_min,
                    "epochs", 65535, threads=threads)
        dt = time.perf_counter() - t0
        votes += float(wl.n) * k
        total_s += dt
        parts.append("%s: %d of %d velocities, %d detections, %.1f s"
                     % (wl.name, k, len(v), wl.n, dt))
    return {"value": votes / total_s, "unit": "votes/s", "cores": threads, "kind": "oracle",
            "sample": "seeded velocity samples over whole catalogs; " + "; ".join(parts)}


def cpu_baseline_night(chips, seconds):
    """The oracle on the first two chips of each style of the night."""
    pick = [c for c in chips if c["style"] == "fast"][:2] + \
        [c for c in chips if c["style"] == "wide"][:2]
    return cpu_baseline([(c["wl"], c["v"], c["n_min"]) for c in pick], seconds)


# --------------------------------------------------------------------------- main

def main():
    from paper_2509_26279_amd import autotune
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="night", choices=["night", "wide", "fast", "tiny"])
    ap.add_argument("--cpu-seconds", type=float, default=16.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--chips", type=int, default=64, help="night: number of chips")
    ap.add_argument("--cache", default=autotune.CACHE, help="tuning cache file (launch shapes per shape class)")
    ap.add_argument("--retune", action="store_true",
                    help="tune every shape class of the workload (library autotuner) and "
                         "store the choices in --cache before the timed run")
    ap.add_argument("--tune-set", choices=["small", "full"], default="small",
                    help="--retune: candidate launch shapes per class")
    ap.add_argument("--no-graph", action="store_true", help="night: eager launches per step")
    ap.add_argument("--ceilings", action="store_true",
                    help="print the measured unit rates (LDS atomics, integer VALU, HBM copy)")
    ap.add_argument("--extract", action="store_true",
                    help="one chip: also time the greedy cluster extraction")
    ap.add_argument("--extract-rounds", type=int, default=0,
                    help="parallel rounds of the extraction (0 default, -1 one take at a time)")
    ap.add_argument("--refine", action="store_true",
                    help="one chip: also time Steps 4-6 over the extraction's clusters")
    ap.add_argument("--refine-starts", type=int, default=500,
                    help="random starts of FAST-MCD per fit (at most 1024)")
    ap.add_argument("--sort-sample", type=int, default=0,
                    help="one chip: also time the sort-by-bin-key path on this many consecutive "
                         "velocities of the grid, against the dense path")
    ap.add_argument("--weighted", choices=["epochs", "detections"], default=None,
                    help="one chip: also time the weighted vote of the same catalog")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; --gpus %d is not supported" % args.gpus,
              file=sys.stderr)
        sys.exit(2)
    if args.ceilings:
        from paper_2509_26279_amd import sas
        c = sas.measure_ceilings()
        c.update({"lds_atomic_peak": LDS_ATOMIC_PEAK, "valu_int32_peak": INT_PEAK_TOPS * 1e12,
                  "valu_int16x2_peak": INT16X2_PEAK_TOPS * 1e12,
                  "hbm_peak_bytes_per_s": HBM_PEAK_GBS * 1e9})
        print(json.dumps({"ceilings": c}), flush=True)
        return
    if args.workload == "night":
        run_night(args)
    else:
        run_chip(args)


if __name__ == "__main__":
    main()
