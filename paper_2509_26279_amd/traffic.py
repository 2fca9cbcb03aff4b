"""HBM traffic of the vote kernel from hardware counters.

Two rocprofv3 passes over the same program, one with FETCH_SIZE and one with
WRITE_SIZE (KiB per dispatch as the counters report them), give the bytes the
vote kernel moves between L2 and HBM.  The same program first runs a plain
device-to-device copy of known size, and the counters' readings for that
copy calibrate them (bytes copied / bytes the counter reports).

    cd /tmp && rocprofv3 --pmc FETCH_SIZE -d OUT/fetch -o fetch --output-format csv \\
        -- python3 -m paper_2509_26279_amd.traffic run wide
    cd /tmp && rocprofv3 --pmc WRITE_SIZE -d OUT/write -o write --output-format csv \\
        -- python3 -m paper_2509_26279_amd.traffic run wide
    python3 -m paper_2509_26279_amd.traffic summarize wide OUT/fetch OUT/write \\
        profiles/traffic_k_vote_dense_wide.json

(run the program with the repository root as the working directory or on
PYTHONPATH).  The summary records the hash of the kernel source it was taken
on; the benchmark reports the traffic only while that hash matches.

Workload "night" votes the batched night once (k_vote_dense_batch, one
dispatch per kernel class): its traffic is the sum over those dispatches,
written to profiles/traffic_k_vote_dense_batch_night.json.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30
KERNEL = "k_vote_dense"


def kernel_source_hash() -> str:
    with open(os.path.join(HERE, "csrc", "vote_dense.hip"), "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def kernel_of(workload: str) -> str:
    return "k_vote_dense_batch" if workload == "night" else KERNEL


def run(workload: str) -> None:
    import torch

    from . import sas, synth
    src = torch.ones(COPY_BYTES // 4, dtype=torch.int32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    dst.copy_(src)  # calibration: COPY_BYTES read, COPY_BYTES written
    torch.cuda.synchronize()
    del src, dst
    if workload == "night":
        from . import night
        chips, _, _ = night.setup()
        b = sas.Batch([(c["plan"], c["x"], c["y"], c["e"]) for c in chips], cand_cap=1 << 21)
        b.vote()
        n = sum(len(b.peaks(k)) for k in range(len(chips)))
        b.close()
        for c in chips:
            c["plan"].close()
        print("traffic run: night, %d candidates" % n, flush=True)
        return
    wl = getattr(synth, "make_" + workload)()
    v = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    plan = sas.Plan(v, wl.t_q16, wl.binw_q8, wl.n_min, wl.extent_q8,
                    count_sat=255 if wl.count_dtype == "u8" else 65535,
                    tuning={"n_det_hint": wl.n})
    s = sas.Search(plan, wl.n, cand_cap=1 << 22)
    x, y, e = s.upload(wl.x_q8, wl.y_q8, wl.epoch)
    s.vote(x, y, e)
    n = len(s.peaks())
    plan.close()
    print("traffic run: %s, %d candidates" % (workload, n), flush=True)


def _rows(d: str):
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        with open(f) as fh:
            yield from csv.DictReader(fh)


def _counter(d: str, name: str, kernel: str = KERNEL):
    """(copy KiB, vote KiB) for one counter: the largest copy-like dispatch
    and the vote kernel's dispatch (the batch kernel: the sum over its
    dispatches, one per kernel class, of the single batched vote)."""
    copy_kib, vote_kib = 0.0, None
    for r in _rows(d):
        if r.get("Counter_Name") != name:
            continue
        k = r.get("Kernel_Name", "")
        val = float(r["Counter_Value"])
        if kernel + "<" in k:
            if kernel == KERNEL:
                vote_kib = val if vote_kib is None else max(vote_kib, val)
            else:
                vote_kib = val + (vote_kib or 0.0)
        elif "copy" in k.lower() or "elementwise" in k.lower():
            copy_kib = max(copy_kib, val)
    return copy_kib, vote_kib


def summarize(workload: str, fetch_dir: str, write_dir: str, out: str) -> dict:
    kernel = kernel_of(workload)
    cf, vf = _counter(fetch_dir, "FETCH_SIZE", kernel)
    cw, vw = _counter(write_dir, "WRITE_SIZE", kernel)
    if not cf or not cw or vf is None or vw is None:
        raise SystemExit("counters missing: copy fetch %s write %s, vote fetch %s write %s"
                         % (cf, cw, vf, vw))
    kf = COPY_BYTES / (cf * 1024.0)
    kw = COPY_BYTES / (cw * 1024.0)
    rec = {
        "kernel": kernel,
        "workload": workload,
        "fetch_kib": vf, "write_kib": vw,
        "copy_bytes": COPY_BYTES, "copy_fetch_kib": cf, "copy_write_kib": cw,
        "fetch_factor": kf, "write_factor": kw,
        "hbm_read_bytes": vf * 1024.0 * kf,
        "hbm_write_bytes": vw * 1024.0 * kw,
        "hbm_bytes_per_launch": vf * 1024.0 * kf + vw * 1024.0 * kw,
        "kernel_source_sha256_16": kernel_source_hash(),
        "command": "rocprofv3 --pmc FETCH_SIZE (then WRITE_SIZE) --output-format csv -- "
                   "python3 -m paper_2509_26279_amd.traffic run %s" % workload,
    }
    with open(out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    return rec


def main(argv):
    if len(argv) >= 2 and argv[0] == "run":
        run(argv[1])
    elif len(argv) == 5 and argv[0] == "summarize":
        print(json.dumps(summarize(*argv[1:]), indent=1))
    else:
        raise SystemExit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
