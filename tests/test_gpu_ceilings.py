"""The measured ceilings the vote kernels' roofline is stated against
(sas_measure_ceilings): each rate is positive and no LDS or HBM rate exceeds
the unit's derived peak (256 CUs x 16 lane-atomics per clock x 2.4 GHz for
the LDS; 8 TB/s for HBM); the LDS atomic add without bank conflicts reaches
most of its peak, which is what makes it the vote's roofline."""
import pytest

from paper_2509_26279_amd import sas

pytestmark = pytest.mark.gpu

LDS_ATOMIC_PEAK = 256 * 16 * 2.4e9
HBM_PEAK = 8.0e12


def test_ceilings_within_the_derived_peaks(gpu):
    c = sas.measure_ceilings()
    print(c, flush=True)
    for k, v in c.items():
        assert v > 0, k
    for k in ("lds_atomic_conflict_free", "lds_atomic_lane_groups"):
        assert c[k] <= 1.02 * LDS_ATOMIC_PEAK, (k, c[k])
    assert c["lds_atomic_conflict_free"] >= 0.5 * LDS_ATOMIC_PEAK
    assert c["hbm_copy_bytes_per_s"] <= HBM_PEAK
    # the packed 16-bit form does two half-operations per lane-op
    assert c["valu_int16x2_ops"] > 0.5 * c["valu_int32_ops"]
