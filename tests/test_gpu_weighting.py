"""Weighted votes against the indicator vote on faint movers (the trade-off
the Conclusions leave open), through the GPU path: at a matched number of
noise candidates, likelihood-weighted votes must find more faint movers and
reach a lower SNR at half completeness."""
import sys

import pytest

from paper_2509_26279_amd import weighting

pytestmark = pytest.mark.gpu


def test_weighted_votes_reach_fainter_movers(gpu):
    r = weighting.compare(log=lambda m: print(m, flush=True, file=sys.stdout))
    print(r, flush=True)
    ind, wtd = r["indicator"], r["weighted"]
    # the operating points are matched on validation chips; on the test
    # chips the noise candidates stay comparable
    assert wtd["noise_candidates"] <= 1.25 * ind["noise_candidates"] + 10
    assert wtd["recall"] > ind["recall"]
    assert wtd["snr50"] < ind["snr50"]
    for a, b in zip(ind["recall_by_snr"], wtd["recall_by_snr"]):
        assert 0.0 <= a <= 1.0 and 0.0 <= b <= 1.0
