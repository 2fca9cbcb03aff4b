"""Learned vetting on the GPU: on the test chips the learned selection must
reach the plain threshold's recall with at least 5x fewer false positives.
Two protocols: fast-style chips (pool at N_pool = 19, 36 training, 12
validation and 12 test chips) and wide-style chips (noise-dominated pools at
the threshold rule's N_pool, about 1e6 candidates over 8 training, 2
validation and 2 test chips).  Judged against injected truth only (the paper
has no learned vetting to compare with)."""
import sys
import time

import pytest

from paper_2509_26279_amd import vetting


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_vetting_gain_fast(gpu):
    t0 = time.time()

    def log(msg):
        print("%6.1fs %s" % (time.time() - t0, msg), file=sys.stderr, flush=True)

    out = vetting.fast_protocol(log=log)
    print(out, flush=True)
    (rec_p, fp_p), (rec_l, fp_l) = out["plain"], out["learned"]
    assert fp_p > 0
    assert rec_l >= rec_p, out
    assert 5 * fp_l <= fp_p, out


@pytest.mark.gpu
@pytest.mark.timeout(600)
def test_vetting_gain_wide(gpu):
    t0 = time.time()

    def log(msg):
        print("%6.1fs %s" % (time.time() - t0, msg), file=sys.stderr, flush=True)

    out = vetting.wide_protocol(log=log)
    print(out, flush=True)
    (rec_p, fp_p), (rec_l, fp_l) = out["plain"], out["learned"]
    total_pool = out["pool_test"]
    assert out["n_pool"] <= 8 and total_pool > 100000  # noise-dominated pools
    assert fp_p > 0
    assert rec_l >= rec_p, out
    assert 5 * fp_l <= fp_p, out
