"""CPU oracle for the catalog shift-and-stack voting transform.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import
anything from this package.  It shares no code with the GPU library
(``paper_2509_26279_amd``) and never imports it; both are fed from the
seeded input generator, which holds none of the method's arithmetic.

Contents
  * ``sas_oracle.c`` - the plain definition of Steps 1-2 (Project, Cluster)
    with the Step-3 threshold read as "report every bin >= N_min" (Sec. 2.1),
    as a per-velocity sort-and-count loop in exact 128-bit integer arithmetic,
    with indicator counts (distinct epochs, detections) or weighted ones (a
    per-detection weight accumulated instead, as the Conclusions suggest);
  * ``brute.py``     - the same definition in exact rationals (tiny inputs);
  * ``grid.py``      - the velocity lattice of Sec. 2 (spacing Delta x / Delta t);
  * ``params.py``    - the threshold rule of Sec. 2.2 (N_min from a target
    number of false candidates);
  * ``features.py``  - candidate features and labels for learned vetting;
  * ``extract.py``   - the greedy cluster extraction of Step 3 (Sec. 2.1);
  * ``refine.py``    - Refine (FAST-MCD robust regression), Gather and their
    iteration, Steps 4-6 (Sec. 2.1, with the regression of Sec. 2);
  * ``mlp_ref.py``   - FP64 reference of the candidate-vetting MLP.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

CAND_DTYPE = np.dtype([("v_idx", "<u4"), ("bx", "<i4"), ("by", "<i4"),
                       ("count", "<u2"), ("flags", "<u2")])


def build(force: bool = False) -> str:
    """Compile the C oracle with gcc (OpenMP) into oracle/liboracle.so."""
    src = os.path.join(_HERE, "sas_oracle.c")
    if force or not os.path.exists(_LIB_PATH) or \
            os.path.getmtime(_LIB_PATH) < os.path.getmtime(src):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC",
                               "-std=gnu11", "-o", tmp, src])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.c_void_p
        lib.oracle_vote.restype = ctypes.c_int64
        lib.oracle_vote.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int32, P,
                                    ctypes.c_int64, P, ctypes.c_int64, ctypes.c_int32,
                                    ctypes.c_int32, ctypes.c_int32, ctypes.c_int32,
                                    P, ctypes.c_int64]
        lib.oracle_histogram.restype = ctypes.c_int
        lib.oracle_histogram.argtypes = [ctypes.c_int64, P, P, P, P, ctypes.c_int32, P,
                                         ctypes.c_int32, ctypes.c_int32, ctypes.c_int64,
                                         ctypes.c_int32, ctypes.c_int64, ctypes.c_int64,
                                         ctypes.c_int64, ctypes.c_int64, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _cat_arrays(x_q8, y_q8, epoch, t_q16):
    x = np.ascontiguousarray(x_q8, dtype=np.int32)
    y = np.ascontiguousarray(y_q8, dtype=np.int32)
    e = np.ascontiguousarray(epoch, dtype=np.uint8)
    t = np.ascontiguousarray(t_q16, dtype=np.int64)
    return x, y, e, t


MODES = {"epochs": 0, "detections": 1, "weighted_epochs": 2, "weighted_detections": 3}


def _weights(mode, weight, n):
    """uint8 weights for the weighted modes (None otherwise)."""
    if MODES[mode] < 2:
        if weight is not None:
            raise ValueError("weights are only taken by the weighted modes")
        return None
    w = np.asarray(weight)
    if w.shape != (n,) or (w.size and (w.min() < 0 or w.max() > 255)):
        raise ValueError("weights: one integer in [0, 255] per detection")
    return np.ascontiguousarray(w, dtype=np.uint8)


def vote(x_q8, y_q8, epoch, t_q16, v_q8, binw_q8, n_min, mode="epochs",
         count_sat=65535, threads=0, weight=None):
    """Candidates (structured array, CAND_DTYPE) ordered by (v_idx, by, bx).
    mode: "epochs", "detections", or the weighted "weighted_epochs" /
    "weighted_detections", which take `weight` (uint8 per detection)."""
    lib = _load()
    x, y, e, t = _cat_arrays(x_q8, y_q8, epoch, t_q16)
    v = np.ascontiguousarray(v_q8, dtype=np.int32).reshape(-1, 2)
    m = MODES[mode]
    w = _weights(mode, weight, x.shape[0])
    cap = 1 << 16
    while True:
        out = np.zeros(cap, dtype=CAND_DTYPE)
        total = lib.oracle_vote(x.shape[0], _ptr(x), _ptr(y), _ptr(e),
                                _ptr(w) if w is not None else None, t.shape[0], _ptr(t),
                                v.shape[0], _ptr(v), int(binw_q8), int(n_min), m,
                                int(count_sat), int(threads), _ptr(out), cap)
        if total < 0:
            raise ValueError("oracle_vote: invalid arguments")
        if total <= cap:
            return out[:total].copy()
        cap = int(total)


def histogram(x_q8, y_q8, epoch, t_q16, u_q8, w_q8, binw_q8, mode, bx0, by0, nbx, nby,
              weight=None):
    """Full histogram of one velocity on a bin window; returns (hist[nby, nbx], outside)."""
    lib = _load()
    x, y, e, t = _cat_arrays(x_q8, y_q8, epoch, t_q16)
    w = _weights(mode, weight, x.shape[0])
    h = np.zeros((nby, nbx), dtype=np.int64)
    outside = np.zeros(1, dtype=np.int64)
    rc = lib.oracle_histogram(x.shape[0], _ptr(x), _ptr(y), _ptr(e),
                              _ptr(w) if w is not None else None, t.shape[0], _ptr(t),
                              int(u_q8), int(w_q8), int(binw_q8),
                              MODES[mode], int(bx0), int(by0),
                              int(nbx), int(nby), _ptr(h), _ptr(outside))
    if rc != 0:
        raise ValueError("oracle_histogram: invalid arguments")
    return h, int(outside[0])
