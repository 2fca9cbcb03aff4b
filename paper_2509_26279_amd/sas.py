"""Python binding of libsas (the C ABI in include/sas.h).

Argument marshalling only: every step of the voting transform runs in the
library's HIP kernels.  PyTorch supplies device memory and streams.  If the
library is missing this module raises; there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsas.so")

SAS_OK = 0
SAS_E_INVALID = -1
SAS_E_NOMEM = -2
SAS_E_OVERFLOW = -3
SAS_E_DEVICE = -4
SAS_E_UNSUPPORTED = -5
SAS_E_WORKSPACE = -6

GRID_SHAPES = {"box": 0, "disk": 1, "annulus": 2, "sector": 3}
MODES = {"epochs": 0, "detections": 1, "weighted_epochs": 2, "weighted_detections": 3}
PATHS = {"auto": 0, "dense": 1, "sort": 2}
ORDERS = {"canonical": 0, "by_count": 1}

N_FEATURES = 32
REFINE_MAX_POINTS = 512
REFINE_STATUS = {0: "converged", 1: "max_rounds", 2: "too_small", 3: "no_start", 4: "too_large",
                 5: "bad_input"}
REFINED_DTYPE = np.dtype([("vx", "<f8"), ("vy", "<f8"), ("x0", "<f8"), ("y0", "<f8"),
                          ("sxx", "<f8"), ("sxy", "<f8"), ("syy", "<f8"),
                          ("n_points", "<i4"), ("n_gathered", "<i4"), ("rounds", "<i4"),
                          ("status", "<i4")])
CAND_DTYPE = np.dtype([("v_idx", "<u4"), ("bx", "<i4"), ("by", "<i4"),
                       ("count", "<u2"), ("flags", "<u2")])


class SasError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (_status_name(status), msg))
        self.status = status


# bits of the vote result's status, with the error sas_peaks returns for each
_DATA_ERRORS = ((1, SAS_E_INVALID, "the catalog holds an epoch index >= n_epochs"),
                (2, SAS_E_INVALID, "a detection lies outside the plan's footprint"),
                (8, SAS_E_DEVICE, "internal error: a tile window exceeded the plan's run table "
                                  "or guard cells"),
                (4, SAS_E_OVERFLOW, "more flagged histogram cells than the plan's refinement "
                                    "list holds"))


class GridSpec(ctypes.Structure):
    _fields_ = [("shape", ctypes.c_int32), ("vmin", ctypes.c_double), ("vmax", ctypes.c_double),
                ("vy_min", ctypes.c_double), ("vy_max", ctypes.c_double),
                ("angle_deg", ctypes.c_double), ("half_width_deg", ctypes.c_double),
                ("binw_q8", ctypes.c_int32), ("span_q16", ctypes.c_int64),
                ("spacing_q8", ctypes.c_int32)]


class Tuning(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("vblock_x", ctypes.c_int32), ("vblock_y", ctypes.c_int32),
                ("groups", ctypes.c_int32), ("stage_cap", ctypes.c_int32),
                ("cell_log2", ctypes.c_int32), ("sort_vblock", ctypes.c_int32),
                ("n_det_hint", ctypes.c_int32), ("coarse_log2", ctypes.c_int32),
                ("refine_cap", ctypes.c_int32), ("packed", ctypes.c_int32),
                ("weight_hint", ctypes.c_int32), ("half_counts", ctypes.c_int32),
                ("prune", ctypes.c_int32)]


class BatchChip(ctypes.Structure):
    _fields_ = [("plan", ctypes.c_void_p), ("x_q8", ctypes.c_void_p), ("y_q8", ctypes.c_void_p),
                ("epoch", ctypes.c_void_p), ("n", ctypes.c_int64), ("cand_dev", ctypes.c_void_p),
                ("cand_cap", ctypes.c_int64), ("res_dev", ctypes.c_void_p)]


class PlanDesc(ctypes.Structure):
    _fields_ = [("v_host", ctypes.c_void_p), ("n_v", ctypes.c_int64),
                ("n_epochs", ctypes.c_int32), ("t_q16", ctypes.c_void_p),
                ("binw_q8", ctypes.c_int32), ("n_min", ctypes.c_int32),
                ("mode", ctypes.c_int32), ("count_sat", ctypes.c_int32),
                ("path", ctypes.c_int32), ("extent_q8", ctypes.c_int32 * 4),
                ("tuning", ctypes.c_void_p)]


class AutotuneTrial(ctypes.Structure):
    _fields_ = [("tuning", Tuning), ("ms", ctypes.c_float), ("status", ctypes.c_int32)]


class PlanInfo(ctypes.Structure):
    _fields_ = [("n_items", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("n_blocks", ctypes.c_int64),
                ("path", ctypes.c_int32), ("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32),
                ("vblock_x", ctypes.c_int32), ("vblock_y", ctypes.c_int32),
                ("cell_log2", ctypes.c_int32), ("coarse_log2", ctypes.c_int32),
                ("mode_variant", ctypes.c_int32), ("n_v", ctypes.c_int64),
                ("groups", ctypes.c_int32), ("hist_x", ctypes.c_int32),
                ("hist_y", ctypes.c_int32), ("stage_cap", ctypes.c_int32),
                ("lds_bytes", ctypes.c_int32), ("packed", ctypes.c_int32),
                ("half_counts", ctypes.c_int32), ("n_tiles_kept", ctypes.c_int64),
                ("n_items_kept", ctypes.c_int64)]


_lib = None

EXPORTS = ["sas_status_string", "sas_last_error", "sas_version", "sas_grid_spacing",
           "sas_build_grid", "sas_plan_create", "sas_plan_destroy", "sas_plan_get_info",
           "sas_plan_set_probe", "sas_plan_set_counter", "sas_batch_set_counter",
           "sas_vote_workspace_size", "sas_vote", "sas_vote_weighted",
           "sas_vote_static", "sas_peaks",
           "sas_threshold_n_min", "sas_batch_workspace_size", "sas_batch_create",
           "sas_batch_destroy", "sas_vote_batch", "sas_batch_set_probe", "sas_features",
           "sas_features_scratch_size", "sas_extract_scratch_size", "sas_extract_clusters",
           "sas_refine_clusters",
           "sas_autotune", "sas_autotune_default_candidates", "sas_autotune_key",
           "sas_autotune_cache_get", "sas_autotune_cache_put",
           "sas_measure_ceilings",
           "sas_mlp_create", "sas_mlp_destroy", "sas_mlp_set_norm", "sas_mlp_get_params",
           "sas_mlp_set_params", "sas_mlp_save", "sas_mlp_load", "sas_mlp_forward", "sas_mlp_grad", "sas_mlp_train_step"]


def load():
    """Load libsas.so (built by ``python -m paper_2509_26279_amd.build``)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libsas.so is not built (%s); run python -m paper_2509_26279_amd.build"
                           % LIB_PATH)
    # torch ships its own HIP runtime; importing it first makes the library
    # bind to that same runtime (one runtime per process, so torch's device
    # memory and streams are the library's too).  Loaded the other way round,
    # torch finds the system runtime already initialised and no device.
    import torch  # noqa: F401
    lib = ctypes.CDLL(LIB_PATH)
    P, I32, I64, SZ = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_size_t
    sig = {
        "sas_status_string": (ctypes.c_char_p, [I32]),
        "sas_last_error": (ctypes.c_char_p, []),
        "sas_version": (ctypes.c_char_p, []),
        "sas_grid_spacing": (I32, [I32, I64, P]),
        "sas_build_grid": (I32, [P, P, I64, P]),
        "sas_plan_create": (I32, [P, P]),
        "sas_plan_destroy": (I32, [P]),
        "sas_plan_get_info": (I32, [P, P]),
        "sas_plan_set_probe": (I32, [P, P, P]),
        "sas_plan_set_counter": (I32, [P, P]),
        "sas_batch_set_counter": (I32, [P, P]),
        "sas_vote_workspace_size": (I32, [P, I64, P]),
        "sas_vote": (I32, [P, P, P, P, I64, P, I64, P, P, SZ, P]),
        "sas_vote_weighted": (I32, [P, P, P, P, P, I64, P, I64, P, P, SZ, P]),
        "sas_vote_static": (I32, [P, P, P, P, I64, P, I64, P, P]),
        "sas_refine_clusters": (I32, [P, P, SZ, P, P, P, I64, P, P, I64, I64, P, I32, I32, P, P,
                                      I32, P, P]),
        "sas_peaks": (I32, [P, P, I64, I32, I64, P, I64, P, P]),
        "sas_threshold_n_min": (I32, [I32, ctypes.c_double, ctypes.c_double, ctypes.c_double,
                                      I32, P]),
        "sas_batch_workspace_size": (I32, [P, I32, P]),
        "sas_batch_create": (I32, [P, I32, P, SZ, P]),
        "sas_batch_destroy": (I32, [P]),
        "sas_vote_batch": (I32, [P, P]),
        "sas_batch_set_probe": (I32, [P, P, P]),
        "sas_features": (I32, [P, P, SZ, I64, P, P, I64, I32, P, SZ, P, P]),
        "sas_features_scratch_size": (I32, [I64, ctypes.POINTER(ctypes.c_size_t)]),
        "sas_extract_scratch_size": (I32, [I64, I64, I64, ctypes.POINTER(ctypes.c_size_t)]),
        "sas_extract_clusters": (I32, [P, P, SZ, I64, P, I64, I64, P, SZ, P, I64, P, P, I32,
                                       P]),
        "sas_autotune": (I32, [P, P, P, P, I64, P, I32, I32, P, P, P]),
        "sas_autotune_default_candidates": (I32, [P, P, I32, P]),
        "sas_autotune_key": (I32, [P, I64, ctypes.c_char_p, I64]),
        "sas_autotune_cache_get": (I32, [ctypes.c_char_p, ctypes.c_char_p, P, P]),
        "sas_autotune_cache_put": (I32, [ctypes.c_char_p, ctypes.c_char_p, P]),
        "sas_measure_ceilings": (I32, [P, P]),
        "sas_mlp_create": (I32, [I64, ctypes.c_uint64, P]),
        "sas_mlp_destroy": (I32, [P]),
        "sas_mlp_set_norm": (I32, [P, P, P]),
        "sas_mlp_get_params": (I32, [P, P, I64, P]),
        "sas_mlp_set_params": (I32, [P, P, I64]),
        "sas_mlp_save": (I32, [P, P, I64, P]),
        "sas_mlp_load": (I32, [P, P, I64]),
        "sas_mlp_forward": (I32, [P, P, I64, P, P]),
        "sas_mlp_grad": (I32, [P, P, P, I64, ctypes.c_float, P, P, P]),
        "sas_mlp_train_step": (I32, [P, P, P, I64, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                     ctypes.c_float, P, P]),
    }
    for name, (res, args) in sig.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def _status_name(s):
    try:
        return load().sas_status_string(s).decode()
    except Exception:  # library not loadable while formatting an error
        return str(s)


def _check(status):
    if status != SAS_OK:
        raise SasError(status, load().sas_last_error().decode())


def version() -> str:
    return load().sas_version().decode()


# --------------------------------------------------------------------------- grid

def grid_spacing(binw_q8: int, span_q16: int) -> int:
    out = ctypes.c_int32()
    _check(load().sas_grid_spacing(int(binw_q8), int(span_q16), ctypes.byref(out)))
    return out.value


def build_grid(shape, vmin=0.0, vmax=0.0, vy_min=0.0, vy_max=0.0, angle_deg=0.0,
               half_width_deg=0.0, binw_q8=1024, span_q16=65536, spacing_q8=0) -> np.ndarray:
    """Velocity lattice as int32 [n, 2] (Q8 px/h) in v_idx order."""
    spec = GridSpec(GRID_SHAPES[shape] if isinstance(shape, str) else int(shape), vmin, vmax,
                    vy_min, vy_max, angle_deg, half_width_deg, int(binw_q8), int(span_q16),
                    int(spacing_q8))
    n = ctypes.c_int64()
    lib = load()
    _check(lib.sas_build_grid(ctypes.byref(spec), None, 0, ctypes.byref(n)))
    out = np.zeros((max(n.value, 1), 2), dtype=np.int32)
    _check(lib.sas_build_grid(ctypes.byref(spec), out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def grid_from_spec(spec, binw_q8: int, span_q16: int) -> np.ndarray:
    """Grid of a ``synth.GridSpec``-like object (shape, vmin, vmax, ...)."""
    return build_grid(spec.shape, spec.vmin, spec.vmax, spec.vy_min, spec.vy_max,
                      spec.angle_deg, spec.half_width_deg, binw_q8, span_q16)


def threshold_n_min(n_epochs: int, mu: float, n_stacks: float, n_false: float = 100.0,
                    mode: str = "epochs") -> int:
    """The threshold rule of Sec. 2.2 (sas_threshold_n_min)."""
    out = ctypes.c_int32()
    _check(load().sas_threshold_n_min(int(n_epochs), float(mu), float(n_stacks), float(n_false),
                                      MODES[mode], ctypes.byref(out)))
    return out.value


# --------------------------------------------------------------------------- plans

def tuning_struct(tuning) -> Tuning:
    """A sas_tuning from a dict of its fields (absent fields 0)."""
    keys = [k for k, _ in Tuning._fields_]
    unknown = sorted(set(tuning) - set(keys))
    if unknown:
        raise ValueError("unknown tuning keys: %s" % ", ".join(unknown))
    return Tuning(*[int(tuning.get(k, 0)) for k in keys])


def tuning_dict(t: Tuning) -> dict:
    """The nonzero fields of a sas_tuning."""
    return {k: int(getattr(t, k)) for k, _ in Tuning._fields_ if getattr(t, k)}


class _Desc:
    """A sas_plan_desc with the arrays it points to kept alive."""

    def __init__(self, velocities, t_q16, binw_q8, n_min, extent_q8, mode="epochs",
                 count_sat=65535, path="auto", tuning=None):
        self.v = np.ascontiguousarray(velocities, dtype=np.int32).reshape(-1, 2)
        self.t = np.ascontiguousarray(t_q16, dtype=np.int64)
        self.tuning = tuning_struct(tuning) if tuning is not None else None
        self.desc = PlanDesc(self.v.ctypes.data, self.v.shape[0], self.t.shape[0],
                             self.t.ctypes.data, int(binw_q8), int(n_min), MODES[mode],
                             int(count_sat), PATHS[path],
                             (ctypes.c_int32 * 4)(*map(int, extent_q8)),
                             ctypes.addressof(self.tuning) if self.tuning is not None else None)


class Plan:
    """A work decomposition for one (velocity set, epochs, parameters, footprint)."""

    def __init__(self, velocities, t_q16, binw_q8, n_min, extent_q8, mode="epochs",
                 count_sat=65535, path="auto", tuning=None):
        lib = load()
        d = _Desc(velocities, t_q16, binw_q8, n_min, extent_q8, mode, count_sat, path, tuning)
        self._v, self._t, self._tuning = d.v, d.t, d.tuning
        self._p = ctypes.c_void_p()
        _check(lib.sas_plan_create(ctypes.byref(d.desc), ctypes.byref(self._p)))
        self.mode = mode
        self.weighted = MODES[mode] >= 2
        self.n_v = self._v.shape[0]
        self.n_epochs = self._t.shape[0]

    @property
    def handle(self):
        return self._p

    def info(self) -> dict:
        inf = PlanInfo()
        _check(load().sas_plan_get_info(self._p, ctypes.byref(inf)))
        return {k: getattr(inf, k) for k, _ in PlanInfo._fields_}

    def set_probe(self, ev_before=None, ev_after=None):
        """Record two torch.cuda.Event objects around the vote kernel of later
        votes with this plan (None, None: off)."""
        h0 = ctypes.c_void_p(ev_before.cuda_event) if ev_before is not None else None
        h1 = ctypes.c_void_p(ev_after.cuda_event) if ev_after is not None else None
        _check(load().sas_plan_set_probe(self._p, h0, h1))

    def set_counter(self, counter=None):
        """Later votes add their LDS atomic vote instructions to `counter`, a
        device int64 tensor of one element (None: off)."""
        _check(load().sas_plan_set_counter(self._p, counter.data_ptr() if counter is not None
                                           else None))

    def workspace_size(self, n: int) -> int:
        out = ctypes.c_size_t()
        _check(load().sas_vote_workspace_size(self._p, int(n), ctypes.byref(out)))
        return out.value

    def close(self):
        if self._p:
            load().sas_plan_destroy(self._p)
            self._p = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# --------------------------------------------------------------------------- autotuner

class Ceilings(ctypes.Structure):
    _fields_ = [("lds_atomic_conflict_free", ctypes.c_double),
                ("lds_atomic_lane_groups", ctypes.c_double),
                ("valu_int32_ops", ctypes.c_double), ("valu_int16x2_ops", ctypes.c_double),
                ("hbm_copy_bytes_per_s", ctypes.c_double)]


def measure_ceilings(stream=None) -> dict:
    """Measured rates of the LDS atomics, integer VALU and HBM (sas_measure_ceilings)."""
    c = Ceilings()
    _check(load().sas_measure_ceilings(ctypes.byref(c), _stream_handle(stream)))
    return {k: float(getattr(c, k)) for k, _ in Ceilings._fields_}


def autotune_key(velocities, t_q16, binw_q8, n_min, extent_q8, n, mode="epochs") -> str:
    """Shape class of a catalog (sas_autotune_key)."""
    d = _Desc(velocities, t_q16, binw_q8, n_min, extent_q8, mode)
    buf = ctypes.create_string_buffer(160)
    _check(load().sas_autotune_key(ctypes.byref(d.desc), int(n), buf, 160))
    return buf.value.decode()


def autotune_default_candidates(velocities, t_q16, binw_q8, n_min, extent_q8, mode="epochs",
                                count_sat=65535, base=None) -> list:
    """The library's built-in candidate tunings around the planner's choice."""
    d = _Desc(velocities, t_q16, binw_q8, n_min, extent_q8, mode, count_sat, "auto", base or {})
    out = (Tuning * 64)()
    n = ctypes.c_int32()
    _check(load().sas_autotune_default_candidates(ctypes.byref(d.desc), out, 64,
                                                  ctypes.byref(n)))
    return [tuning_dict(out[k]) for k in range(n.value)]


def autotune(velocities, t_q16, binw_q8, n_min, extent_q8, x, y, epoch, cands, reps=3,
             mode="epochs", count_sat=65535, stream=None):
    """sas_autotune over the candidate tunings (dicts): (best tuning dict,
    [(tuning dict, ms or None, status)])."""
    d = _Desc(velocities, t_q16, binw_q8, n_min, extent_q8, mode, count_sat)
    arr = (Tuning * len(cands))(*[tuning_struct(c) for c in cands])
    trials = (AutotuneTrial * len(cands))()
    best = Tuning()
    _check(load().sas_autotune(ctypes.byref(d.desc), x.data_ptr(), y.data_ptr(), epoch.data_ptr(),
                               int(x.numel()), arr, len(cands), int(reps), trials,
                               ctypes.byref(best), _stream_handle(stream)))
    table = [(tuning_dict(t.tuning), float(t.ms) if t.ms >= 0 else None, int(t.status))
             for t in trials]
    return tuning_dict(best), table


def autotune_cache_get(path: str, key: str):
    """The cached tuning dict of a shape class, or None."""
    t = Tuning()
    found = ctypes.c_int32()
    _check(load().sas_autotune_cache_get(path.encode(), key.encode(), ctypes.byref(t),
                                         ctypes.byref(found)))
    return tuning_dict(t) if found.value else None


def autotune_cache_put(path: str, key: str, tuning: dict) -> None:
    t = tuning_struct(tuning)
    _check(load().sas_autotune_cache_put(path.encode(), key.encode(), ctypes.byref(t)))


def _stream_handle(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def vote(plan: Plan, x, y, epoch, cand, res, workspace, stream=None, weight=None):
    """Enqueue sas_vote (sas_vote_weighted when `weight` is given).  x, y:
    int32, epoch and weight: uint8 device tensors; cand: device tensor of
    >= 16*cap bytes; res: 16-byte device tensor; workspace: device uint8
    tensor."""
    n = int(x.numel())
    cap = cand.numel() * cand.element_size() // 16
    ws = workspace.numel() * workspace.element_size()
    if weight is None:
        _check(load().sas_vote(plan.handle, x.data_ptr(), y.data_ptr(), epoch.data_ptr(), n,
                               cand.data_ptr(), cap, res.data_ptr(), workspace.data_ptr(), ws,
                               _stream_handle(stream)))
    else:
        if weight.numel() != n:
            raise ValueError("one weight per detection")
        _check(load().sas_vote_weighted(plan.handle, x.data_ptr(), y.data_ptr(),
                                        epoch.data_ptr(), weight.data_ptr(), n,
                                        cand.data_ptr(), cap, res.data_ptr(),
                                        workspace.data_ptr(), ws, _stream_handle(stream)))


STATIC_SCRATCH_BYTES = 64 * 1024 * 1024


def vote_static(plan: Plan, x, y, epoch, cand, res, stream=None):
    """Enqueue sas_vote_static: sas_vote with the library's static per-GPU
    scratch array in place of a workspace (no allocation)."""
    n = int(x.numel())
    cap = cand.numel() * cand.element_size() // 16
    _check(load().sas_vote_static(plan.handle, x.data_ptr(), y.data_ptr(), epoch.data_ptr(), n,
                                  cand.data_ptr(), cap, res.data_ptr(), _stream_handle(stream)))


def peaks(cand, res, order="canonical", top_k=0, stream=None, out=None):
    """Synchronise and return the candidates as a CAND_DTYPE array.  out: an
    optional host CAND_DTYPE array of at least the buffer's capacity, used
    as the landing area (kept by Search across calls)."""
    lib = load()
    cap = cand.numel() * cand.element_size() // 16
    n = ctypes.c_int64()
    if out is None or out.dtype != CAND_DTYPE or out.shape[0] < max(cap, 1):
        out = np.empty(max(cap, 1), dtype=CAND_DTYPE)
    _check(lib.sas_peaks(cand.data_ptr(), res.data_ptr(), cap, ORDERS[order], int(top_k),
                         out.ctypes.data, out.shape[0], ctypes.byref(n), _stream_handle(stream)))
    return out[:n.value].copy()


def features_scratch_size(n_cand: int) -> int:
    """Device scratch bytes sas_features needs for n_cand candidates."""
    out = ctypes.c_size_t(0)
    _check(load().sas_features_scratch_size(int(n_cand), ctypes.byref(out)))
    return int(out.value)


class Search:
    """Device buffers for repeated searches of catalogs with one plan."""

    def __init__(self, plan: Plan, n_max: int, cand_cap: int = 1 << 20, device="cuda"):
        import torch
        self.plan = plan
        self.device = device
        self.n_max = int(n_max)
        self.ws = torch.empty(max(plan.workspace_size(self.n_max), 256), dtype=torch.uint8,
                              device=device)
        self.cand = torch.empty((max(int(cand_cap), 1), 4), dtype=torch.int32, device=device)
        self.res = torch.zeros(4, dtype=torch.int32, device=device)
        self._out = None  # host landing array of peaks()

    def upload(self, x_q8, y_q8, epoch, weight=None):
        """Device copies of a catalog (and of its weights, when given)."""
        import torch
        x = torch.as_tensor(np.ascontiguousarray(x_q8, dtype=np.int32)).to(self.device)
        y = torch.as_tensor(np.ascontiguousarray(y_q8, dtype=np.int32)).to(self.device)
        e = torch.as_tensor(np.ascontiguousarray(epoch, dtype=np.uint8)).to(self.device)
        if weight is None:
            return x, y, e
        w = np.asarray(weight)
        if w.size and (w.min() < 0 or w.max() > 255):
            raise ValueError("weights must lie in [0, 255]")
        return x, y, e, torch.as_tensor(np.ascontiguousarray(w, dtype=np.uint8)).to(self.device)

    def vote(self, x, y, e, w=None, stream=None):
        """Vote a device catalog; a weighted plan takes the weights w."""
        if x.numel() > self.n_max:
            raise ValueError("catalog larger than this Search was sized for")
        if self.plan.weighted != (w is not None):
            raise ValueError("weights are given exactly when the plan counts weights")
        vote(self.plan, x, y, e, self.cand, self.res, self.ws, stream, weight=w)

    def peaks(self, order="canonical", top_k=0, stream=None):
        if self._out is None:
            self._out = np.empty(self.cand.shape[0], dtype=CAND_DTYPE)
        return peaks(self.cand, self.res, order, top_k, stream, out=self._out)

    def _complete_vote(self) -> int:
        """Number of candidates of the last vote, after the checks sas_peaks
        makes: data errors in its status, and more candidates than the buffer
        holds, raise SasError."""
        r = self.result()
        for bit, code, msg in _DATA_ERRORS:
            if r["status"] & bit:
                raise SasError(code, "the last vote: " + msg)
        if r["n_cand"] > self.cand.shape[0]:
            raise SasError(SAS_E_OVERFLOW, "the last vote found %d candidates, more than the "
                                           "buffer's %d" % (r["n_cand"], self.cand.shape[0]))
        return r["n_cand"]

    def result(self) -> dict:
        """The device-side vote result (synchronises): n_cand, status, n_spilled."""
        r = self.res.cpu().numpy().view(np.int32)
        n_cand = int(r[0].astype(np.int64) | (r[1].astype(np.int64) << 32))
        return {"n_cand": n_cand, "status": int(r[2]), "n_spilled": int(r[3])}

    def extract(self, n: int, member_cap: int = 0, cluster_cap: int = 0, rounds: int = 0,
                stream=None):
        """Step 3 (greedy cluster extraction) over the candidates left in the
        device buffer by the last vote of an n-detection catalog.  Returns
        (clusters as CAND_DTYPE in extraction order, int32 [n] cluster of each
        detection or -1).  rounds: parallel rounds before the one-at-a-time
        finish (0 default, -1 none).  Synchronises; grows member_cap once if
        the contributor lists did not fit."""
        import torch
        k = self._complete_vote()
        dev = self.cand.device
        member_cap = int(member_cap or 64 * k + int(n))
        cluster_cap = int(cluster_cap or max(k, 1))
        for _ in range(2):
            nb = ctypes.c_size_t(0)
            _check(load().sas_extract_scratch_size(int(n), k, member_cap, ctypes.byref(nb)))
            scratch = torch.empty(max(nb.value, 1), dtype=torch.uint8, device=dev)
            clusters = torch.empty((max(cluster_cap, 1), 16), dtype=torch.uint8, device=dev)
            owner = torch.empty(max(int(n), 1), dtype=torch.int32, device=dev)
            res = torch.zeros(24, dtype=torch.uint8, device=dev)
            _check(load().sas_extract_clusters(self.plan.handle, self.ws.data_ptr(),
                                               self.ws.numel() * self.ws.element_size(), int(n),
                                               self.cand.data_ptr(), k, member_cap,
                                               scratch.data_ptr(), nb.value, clusters.data_ptr(),
                                               cluster_cap, owner.data_ptr(), res.data_ptr(),
                                               int(rounds), _stream_handle(stream)))
            rr = res.cpu().numpy()
            n_clusters = int(rr[0:8].view(np.int64)[0])
            n_members = int(rr[8:16].view(np.int64)[0])
            status = int(rr[16:20].view(np.int32)[0])
            if status & 1:  # the contributor lists did not fit: once more, sized
                member_cap = n_members
                continue
            if status & 2:
                raise SasError(-3, "sas_extract_clusters: %d clusters, cluster_cap %d"
                               % (n_clusters, cluster_cap))
            recs = clusters[:n_clusters].cpu().numpy().view(CAND_DTYPE).reshape(-1).copy()
            return recs, owner[:int(n)].cpu().numpy()
        raise SasError(-3, "sas_extract_clusters: contributor lists exceed %d" % member_cap)

    def features(self, n: int, snr=None, spacing_q8: int = 0, stream=None):
        """Features of the candidates left in the device buffer by the last
        vote of an n-detection catalog: (records as CAND_DTYPE in buffer
        order, float32 [n_cand, 32]).  snr: device float tensor [n] or None;
        spacing_q8: the velocity grid's lattice spacing (0: no neighbour
        features)."""
        import torch
        k = self._complete_vote()
        feat = torch.empty((max(k, 1), N_FEATURES), dtype=torch.float32, device=self.cand.device)
        nb = features_scratch_size(k) if spacing_q8 else 0
        scratch = torch.empty(max(nb, 1), dtype=torch.uint8, device=self.cand.device)
        _check(load().sas_features(self.plan.handle, self.ws.data_ptr(),
                                   self.ws.numel() * self.ws.element_size(), int(n),
                                   snr.data_ptr() if snr is not None else None,
                                   self.cand.data_ptr(), k, int(spacing_q8),
                                   scratch.data_ptr(), nb, feat.data_ptr(),
                                   _stream_handle(stream)))
        recs = self.cand[:k].cpu().numpy().view(CAND_DTYPE).reshape(-1)
        return recs.copy(), feat[:k].cpu().numpy()

    def refine(self, x, y, e, clusters, starts, radius_q8: int = 0, gather_cap: int = 512,
               subsets: bool = True, stream=None):
        """Steps 4-6 for clusters of the catalog last voted (device tensors
        x, y, e): clusters is a list of catalog-index arrays, starts the
        uint32 [k, 4] draws of the FAST-MCD starts.  Returns (records as
        REFINED_DTYPE, gathered sets, MCD subsets) with the sets as sorted
        catalog-index arrays."""
        import torch
        lens = np.array([len(c) for c in clusters], dtype=np.int64)
        first = np.zeros(len(clusters) + 1, dtype=np.int32)
        first[1:] = np.cumsum(lens)
        members = (np.concatenate([np.asarray(c, dtype=np.int32) for c in clusters])
                   if len(clusters) and lens.sum() else np.zeros(1, np.int32))
        st = np.ascontiguousarray(starts, dtype=np.uint32).reshape(-1, 4)
        dev = self.cand.device
        first_d = torch.as_tensor(first).to(dev)
        mem_d = torch.as_tensor(members).to(dev)
        st_d = torch.as_tensor(st.view(np.int32)).to(dev)
        k = max(len(clusters), 1)
        out = torch.zeros((k, REFINED_DTYPE.itemsize), dtype=torch.uint8, device=dev)
        gath = torch.zeros((k, gather_cap), dtype=torch.int32, device=dev)
        sub = (torch.zeros((k, REFINE_MAX_POINTS), dtype=torch.int32, device=dev)
               if subsets else None)
        _check(load().sas_refine_clusters(
            self.plan.handle, self.ws.data_ptr(), self.ws.numel() * self.ws.element_size(),
            x.data_ptr(), y.data_ptr(), e.data_ptr(), int(x.numel()), first_d.data_ptr(),
            mem_d.data_ptr(), int(lens.sum()), len(clusters), st_d.data_ptr(), st.shape[0],
            int(radius_q8), out.data_ptr(), gath.data_ptr(), int(gather_cap),
            sub.data_ptr() if sub is not None else None, _stream_handle(stream)))
        recs = out.cpu().numpy().view(REFINED_DTYPE).reshape(-1)[:len(clusters)].copy()
        g = gath.cpu().numpy()
        gathered = [g[i, :min(int(r["n_gathered"]), gather_cap)].copy() if r["rounds"] > 0
                    else np.zeros(0, np.int32) for i, r in enumerate(recs)]
        subs = None
        if sub is not None:
            sm = sub.cpu().numpy()
            subs = [sm[i, :int(r["n_points"])].copy() if r["rounds"] > 0
                    else np.zeros(0, np.int32) for i, r in enumerate(recs)]
        return recs, gathered, subs

    def run(self, x_q8, y_q8, epoch, order="canonical", top_k=0, weight=None):
        """Upload, vote (with the weights of a weighted plan) and collect."""
        dev = self.upload(x_q8, y_q8, epoch, weight)
        self.vote(*dev)
        return self.peaks(order, top_k)


class Batch:
    """Many catalogs voted by one persistent launch per kernel class.

    chips: list of (plan, x, y, epoch) with device tensors; each chip gets
    its own candidate buffer and result."""

    def __init__(self, chips, cand_cap: int = 1 << 18, device="cuda"):
        import torch
        lib = load()
        self.plans = [c[0] for c in chips]
        self.tensors = []
        self.cand = []
        self.res = []
        arr = (BatchChip * len(chips))()
        for k, (plan, x, y, e) in enumerate(chips):
            cand = torch.empty((max(int(cand_cap), 1), 4), dtype=torch.int32, device=device)
            res = torch.zeros(4, dtype=torch.int32, device=device)
            self.tensors.append((x, y, e))
            self.cand.append(cand)
            self.res.append(res)
            arr[k] = BatchChip(plan.handle.value, x.data_ptr(), y.data_ptr(), e.data_ptr(),
                               int(x.numel()), cand.data_ptr(), cand.shape[0], res.data_ptr())
        self._arr = arr
        size = ctypes.c_size_t()
        _check(lib.sas_batch_workspace_size(ctypes.byref(arr), len(chips), ctypes.byref(size)))
        self.ws = torch.empty(max(size.value, 256), dtype=torch.uint8, device=device)
        self._b = ctypes.c_void_p()
        _check(lib.sas_batch_create(ctypes.byref(arr), len(chips), self.ws.data_ptr(),
                                    self.ws.numel(), ctypes.byref(self._b)))

    def vote(self, stream=None):
        _check(load().sas_vote_batch(self._b, _stream_handle(stream)))

    def set_probe(self, ev_before=None, ev_after=None):
        h0 = ctypes.c_void_p(ev_before.cuda_event) if ev_before is not None else None
        h1 = ctypes.c_void_p(ev_after.cuda_event) if ev_after is not None else None
        _check(load().sas_batch_set_probe(self._b, h0, h1))

    def set_counter(self, counter=None):
        """Later votes add their LDS atomic vote instructions to `counter`, a
        device int64 tensor of one element (None: off)."""
        _check(load().sas_batch_set_counter(self._b, counter.data_ptr() if counter is not None
                                            else None))

    def peaks(self, k: int, order="canonical", top_k=0, stream=None):
        return peaks(self.cand[k], self.res[k], order, top_k, stream)

    def close(self):
        if self._b:
            load().sas_batch_destroy(self._b)
            self._b = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


MLP_PARAMS = 20865


class MLP:
    """The vetting network (sas_mlp_*): 32 -> 128 -> 128 -> 1 on bf16 MFMA."""

    def __init__(self, max_batch: int = 4096, seed: int = 0, device="cuda"):
        import torch
        self.device = device
        self.max_batch = int(max_batch)
        self._m = ctypes.c_void_p()
        _check(load().sas_mlp_create(self.max_batch, ctypes.c_uint64(seed), ctypes.byref(self._m)))
        self._loss = torch.zeros(1, dtype=torch.float32, device=device)

    def set_norm(self, mean, std):
        m = np.ascontiguousarray(mean, dtype=np.float32)
        s = np.ascontiguousarray(std, dtype=np.float32)
        _check(load().sas_mlp_set_norm(self._m, m.ctypes.data, s.ctypes.data))

    def params(self) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        n = ctypes.c_int64()
        _check(load().sas_mlp_get_params(self._m, out.ctypes.data, MLP_PARAMS, ctypes.byref(n)))
        return out

    def set_params(self, p):
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(load().sas_mlp_set_params(self._m, p.ctypes.data, p.shape[0]))

    def save(self) -> bytes:
        """Checkpoint (sas_mlp_save): header, masters, AdamW moments, norm."""
        n = ctypes.c_int64()
        lib = load()
        st = lib.sas_mlp_save(self._m, None, 0, ctypes.byref(n))
        if st not in (SAS_OK, SAS_E_OVERFLOW):
            _check(st)
        buf = ctypes.create_string_buffer(n.value)
        _check(lib.sas_mlp_save(self._m, buf, n.value, ctypes.byref(n)))
        return buf.raw[:n.value]

    def load(self, blob: bytes):
        """Restore a checkpoint written by save() (sas_mlp_load)."""
        buf = ctypes.create_string_buffer(bytes(blob), len(blob))
        _check(load().sas_mlp_load(self._m, buf, len(blob)))

    def forward(self, x, stream=None):
        import torch
        out = torch.empty(x.shape[0], dtype=torch.float32, device=x.device)
        _check(load().sas_mlp_forward(self._m, x.data_ptr(), x.shape[0], out.data_ptr(),
                                      _stream_handle(stream)))
        return out

    def grad(self, x, y, pos_weight=1.0, stream=None):
        import torch
        g = torch.empty(MLP_PARAMS, dtype=torch.float32, device=x.device)
        _check(load().sas_mlp_grad(self._m, x.data_ptr(), y.data_ptr(), x.shape[0],
                                   float(pos_weight), self._loss.data_ptr(), g.data_ptr(),
                                   _stream_handle(stream)))
        return self._loss, g

    def train_step(self, x, y, pos_weight=1.0, lr=1e-3, betas=(0.9, 0.999), eps=1e-8,
                   weight_decay=0.01, stream=None):
        _check(load().sas_mlp_train_step(self._m, x.data_ptr(), y.data_ptr(), x.shape[0],
                                         float(pos_weight), float(lr), float(betas[0]),
                                         float(betas[1]), float(eps), float(weight_decay),
                                         self._loss.data_ptr(), _stream_handle(stream)))
        return self._loss

    def close(self):
        if self._m:
            load().sas_mlp_destroy(self._m)
            self._m = ctypes.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
