"""Host-side checks of the C ABI that need no GPU: the library loads, every
symbol that include/sas.h declares is exported, the grid builder matches
the oracle's grid, and argument errors are caught before any device work."""
import ctypes
import dataclasses
import os
import re

import numpy as np
import pytest

from oracle import grid as ogrid
from paper_2509_26279_amd import sas, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    txt = open(os.path.join(ROOT, "include", "sas.h")).read()
    return sorted(set(re.findall(r"^\w[\w\s\*]*?\b(sas_\w+)\s*\(", txt, re.M)))


def _exported():
    """Names of the sas_* functions the built library exports (dynamic symbols)."""
    import subprocess
    out = subprocess.run(["nm", "-D", "--defined-only", sas.LIB_PATH], capture_output=True,
                         text=True, check=True).stdout
    return sorted({ln.split()[-1] for ln in out.splitlines()
                   if len(ln.split()) == 3 and ln.split()[1] == "T"
                   and ln.split()[-1].startswith("sas_")})


def test_library_exports_every_declared_symbol():
    lib = sas.load()
    names = _declared()
    assert "sas_vote" in names and "sas_peaks" in names and "sas_build_grid" in names
    for n in names:
        assert hasattr(lib, n), n
    # the header, the library's exported functions and the binding's list agree
    assert set(_exported()) == set(names), sorted(set(_exported()) ^ set(names))
    assert set(sas.EXPORTS) == set(names), sorted(set(sas.EXPORTS) ^ set(names))
    assert "gfx950" in sas.version()


@pytest.mark.parametrize("maker", [synth.make_tiny, synth.make_wide, synth.make_fast])
def test_grid_matches_oracle(maker):
    wl = maker()
    spec = dataclasses.asdict(wl.grid)
    s = ogrid.spacing_q8(wl.binw_q8, wl.span_q16)
    assert sas.grid_spacing(wl.binw_q8, wl.span_q16) == s
    a = sas.grid_from_spec(wl.grid, wl.binw_q8, wl.span_q16)
    b = ogrid.build_grid(spec, s)
    assert np.array_equal(a, b)


@pytest.mark.parametrize("shape,kw", [
    ("annulus", dict(vmin=100.0, vmax=300.0)),
    ("sector", dict(vmin=5.0, vmax=60.0, angle_deg=37.0, half_width_deg=20.0)),
    ("sector", dict(vmin=0.0, vmax=33.3, angle_deg=-90.0, half_width_deg=45.0)),
    ("box", dict(vmin=-3.3, vmax=17.9, vy_min=-40.0, vy_max=-2.0)),
    ("disk", dict(vmax=77.7)),
])
def test_grid_shapes_match_oracle(shape, kw):
    for binw, span in ((1024, 65536 * 3), (333, 99999), (4096, 131072)):
        s = ogrid.spacing_q8(binw, span)
        spec = dict(shape=shape, vmin=0.0, vmax=0.0, vy_min=0.0, vy_max=0.0, angle_deg=0.0,
                    half_width_deg=0.0)
        spec.update(kw)
        a = sas.build_grid(shape, binw_q8=binw, span_q16=span, **kw)
        b = ogrid.build_grid(spec, s)
        assert np.array_equal(a, b), (shape, binw, span)


def test_grid_two_call_protocol():
    lib = sas.load()
    spec = sas.GridSpec(1, 0, 10.0, 0, 0, 0, 0, 1024, 65536, 0)
    n = ctypes.c_int64()
    assert lib.sas_build_grid(ctypes.byref(spec), None, 0, ctypes.byref(n)) == sas.SAS_OK
    buf = np.zeros((2, 2), np.int32)
    rc = lib.sas_build_grid(ctypes.byref(spec), buf.ctypes.data, 2, ctypes.byref(n))
    assert rc == sas.SAS_E_OVERFLOW and n.value > 2
    spec.shape = 3
    spec.half_width_deg = 95.0
    assert lib.sas_build_grid(ctypes.byref(spec), None, 0, ctypes.byref(n)) == sas.SAS_E_INVALID


def _plan_error(**over):
    kw = dict(velocities=np.zeros((4, 2), np.int32), t_q16=np.arange(5) * 65536,
              binw_q8=1024, n_min=3, extent_q8=(0, 1 << 16, 0, 1 << 16))
    kw.update(over)
    with pytest.raises(sas.SasError) as ei:
        sas.Plan(**kw)
    return ei.value.status


@pytest.mark.parametrize("over,status", [
    (dict(binw_q8=0), sas.SAS_E_INVALID),
    (dict(binw_q8=1000), sas.SAS_E_UNSUPPORTED),
    (dict(n_min=0), sas.SAS_E_INVALID),
    (dict(t_q16=np.zeros(0, np.int64)), sas.SAS_E_INVALID),
    (dict(t_q16=np.arange(257) * 100), sas.SAS_E_INVALID),
    (dict(t_q16=np.array([0, 1 << 31])), sas.SAS_E_INVALID),
    (dict(extent_q8=(5, 5, 0, 10)), sas.SAS_E_INVALID),
    (dict(extent_q8=(0, 1 << 30, 0, 10)), sas.SAS_E_INVALID),
    (dict(count_sat=1000), sas.SAS_E_INVALID),
    (dict(velocities=np.array([[1 << 29, 0]], np.int32), t_q16=np.array([0, 1 << 30])),
     sas.SAS_E_UNSUPPORTED),
    (dict(mode="weighted_epochs", path="sort"), sas.SAS_E_UNSUPPORTED),
    (dict(mode="weighted_detections", path="sort"), sas.SAS_E_UNSUPPORTED),
    (dict(tuning=dict(half_counts=2)), sas.SAS_E_INVALID),
    (dict(tuning=dict(half_counts=-2)), sas.SAS_E_INVALID),
])
def test_plan_argument_errors(over, status):
    assert _plan_error(**over) == status


@pytest.mark.parametrize("n_epochs,mu,n_stacks,mode", [
    (60, 0.0916, 1.23e6 * 32768, "epochs"),
    (100, 0.0057, 84351 * 524288, "epochs"),
    (20, 0.02, 441 * 16384, "epochs"),
    (40, 0.3, 1e9, "epochs"),
    (120, 0.001, 1e11, "epochs"),
    (60, 0.0916, 1e10, "detections"),
    (100, 0.0057, 4.4e10, "detections"),
])
def test_threshold_rule_matches_oracle(n_epochs, mu, n_stacks, mode):
    from oracle import params as oparams
    assert sas.threshold_n_min(n_epochs, mu, n_stacks, 100.0, mode) == \
        oparams.choose_n_min(n_epochs, mu, n_stacks, 100.0, mode)


def test_threshold_rule_edges():
    from oracle import params as oparams
    with pytest.raises(sas.SasError):
        sas.threshold_n_min(0, 0.1, 1e6)
    # every count up to E is too frequent: the rule answers E + 1, unreachable
    assert sas.threshold_n_min(10, 5.0, 1e30) == oparams.choose_n_min(10, 5.0, 1e30) == 11
    assert sas.threshold_n_min(10, 0.0, 1e30) == 1


def test_batch_argument_errors():
    lib = sas.load()
    size = ctypes.c_size_t()
    assert lib.sas_batch_workspace_size(None, 0, ctypes.byref(size)) == sas.SAS_E_INVALID
    arr = (sas.BatchChip * 1)()
    assert lib.sas_batch_workspace_size(ctypes.byref(arr), 1, ctypes.byref(size)) == \
        sas.SAS_E_INVALID  # null plan


def test_autotune_classes_and_cache(tmp_path):
    from paper_2509_26279_amd import autotune
    v = np.zeros((84351, 2), np.int32)
    t100 = np.arange(100) * 262144 // 99  # 4 h in Q16
    ext = (0, 2048 * 256, 0, 4096 * 256)
    k1 = autotune.shape_class(v, t100, 1024, 25, ext, 309460)
    assert k1 == "b1024_s256_E64_n262144_V65536_m0", k1
    t127 = np.arange(127) * 262144 // 126  # same span, more epochs in the same octave
    assert k1 == autotune.shape_class(v, t127, 1024, 25, ext, 300000)
    assert k1 != autotune.shape_class(v, np.arange(128) * 262144 // 127, 1024, 25, ext, 300000)
    assert k1 != autotune.shape_class(v, t100, 4096, 25, ext, 309460)
    assert k1 != autotune.shape_class(v[:1000], t100, 1024, 25, ext, 309460)
    assert k1 != autotune.shape_class(v, t100, 1024, 25, ext, 309460, mode="detections")
    p = str(tmp_path / "tune.txt")
    assert autotune.cached(k1, p) is None  # no file: empty cache
    autotune.store(k1, {"groups": 1, "tile_x": 12}, p)
    autotune.store("b4096_other", {}, p)
    autotune.store(k1, {"groups": 2, "n_det_hint": 5}, p)  # replaces the line
    assert autotune.cached(k1, p) == {"groups": 2, "n_det_hint": 5}
    assert autotune.cached("b4096_other", p) == {}
    assert open(p).read().splitlines() == ["b1024_s256_E64_n262144_V65536_m0 groups=2 "
                                           "n_det_hint=5", "b4096_other"]
    with open(p, "a") as f:
        f.write("bad_line groups=1 nonsense=3\n")
    with pytest.raises(sas.SasError):
        autotune.cached("bad_line", p)


def test_refine_extract_weighted_argument_errors():
    """Argument checks that run before any device work (no GPU needed)."""
    lib = sas.load()
    # no plan
    assert lib.sas_refine_clusters(None, None, 0, None, None, None, 0, None, None, 0, 0, None,
                                   1, 0, None, None, 0, None, None) == sas.SAS_E_INVALID
    assert lib.sas_vote_weighted(None, None, None, None, None, 0, None, 0, None, None, 0,
                                 None) == sas.SAS_E_INVALID
    assert lib.sas_extract_clusters(None, None, 0, 0, None, 0, 0, None, 0, None, 0, None, None,
                                    0, None) == sas.SAS_E_INVALID


def test_unknown_tuning_key_rejected():
    with pytest.raises(ValueError):
        sas.Plan(np.zeros((1, 2), np.int32), np.arange(4) * 1000, 1024, 2, (0, 4096, 0, 4096),
                 tuning=dict(half_count=1))
