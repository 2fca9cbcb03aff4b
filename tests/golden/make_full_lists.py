"""Write the oracle's complete candidate lists of the wide and fast workloads.

    python tests/golden/make_full_lists.py [wide|fast ...]

Calls only ``oracle/`` (the plain definition of Steps 1-2 with the threshold
of Step 3, Sec. 2.1) on inputs from the seeded generator.  Each output file
``tests/golden/full_<workload>.txt`` holds a header of ``#`` lines (the
workload, its sizes, a SHA-256 of the generated inputs and of the records)
and then one record per line, ``v_idx bx by count flags``, in the canonical
order (v_idx, by, bx).  The GPU parity tests compare every record of the
whole-grid search with these lists, after checking that the generator gave
the same inputs (same input hash).

Run time on 8 host cores: about 5 min (wide, 2.6e10 votes) and about 45 min
(fast, 2.3e11 votes).
"""
from __future__ import annotations

import dataclasses
import hashlib
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from oracle import grid as ogrid  # noqa: E402
from paper_2509_26279_amd import synth  # noqa: E402

# count saturation of each workload's reported counts (u8 / u16 counts)
SAT = {"wide": 255, "fast": 65535}


def input_hash(wl, v) -> str:
    h = hashlib.sha256()
    for a in (wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def records_hash(c) -> str:
    h = hashlib.sha256()
    for k in ("v_idx", "bx", "by", "count", "flags"):
        h.update(np.ascontiguousarray(c[k]).astype("<i8").tobytes())
    return h.hexdigest()


def path_of(name: str) -> str:
    return os.path.join(HERE, "full_%s.txt" % name)


def workload(name: str):
    wl = {"wide": synth.make_wide, "fast": synth.make_fast}[name]()
    v = ogrid.build_grid(dataclasses.asdict(wl.grid),
                         ogrid.spacing_q8(wl.binw_q8, wl.span_q16))
    return wl, v


def write(name: str) -> None:
    wl, v = workload(name)
    t0 = time.time()
    c = oracle.vote(wl.x_q8, wl.y_q8, wl.epoch, wl.t_q16, v, wl.binw_q8, wl.n_min,
                    "epochs", SAT[name])
    dt = time.time() - t0
    lines = ["# oracle candidate list, whole grid, mode epochs",
             "# workload %s seed %d" % (name, wl.seed),
             "# n %d n_v %d binw_q8 %d n_min %d count_sat %d" % (
                 wl.n, len(v), wl.binw_q8, wl.n_min, SAT[name]),
             "# input_sha256 %s" % input_hash(wl, v),
             "# records %d records_sha256 %s" % (len(c), records_hash(c)),
             "# columns v_idx bx by count flags"]
    lines += ["%d %d %d %d %d" % (r["v_idx"], r["bx"], r["by"], r["count"], r["flags"])
              for r in c]
    tmp = path_of(name) + ".tmp"
    with open(tmp, "w") as f:
        f.write("\n".join(lines) + "\n")
    os.replace(tmp, path_of(name))
    print("%s: %d records in %.0f s -> %s" % (name, len(c), dt, path_of(name)), flush=True)


def read(name: str):
    """(header dict, structured array of records) of a stored list."""
    head = {}
    rows = []
    with open(path_of(name)) as f:
        for line in f:
            if line.startswith("#"):
                parts = line[1:].split()
                for i in range(0, len(parts) - 1, 2):
                    head[parts[i]] = parts[i + 1]
            elif line.strip():
                rows.append([int(t) for t in line.split()])
    a = np.asarray(rows, dtype=np.int64).reshape(-1, 5)
    c = np.zeros(len(a), dtype=oracle.CAND_DTYPE)
    for i, k in enumerate(("v_idx", "bx", "by", "count", "flags")):
        c[k] = a[:, i]
    return head, c


if __name__ == "__main__":
    for name in (sys.argv[1:] or ["wide", "fast"]):
        write(name)
