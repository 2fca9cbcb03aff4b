"""Host-side pieces of the weighted-vote comparison and the faint-mover
generator (CPU): the SNR at half completeness, the selection count, the
likelihood weights and the physics of the faint catalogs."""
import numpy as np
import pytest

from paper_2509_26279_amd import synth, weighting


def test_snr50_interpolates_between_bin_centres():
    bins = np.array([1.0, 2.0, 3.0, 4.0])
    snr = np.array([1.5] * 4 + [2.5] * 4 + [3.5] * 4)
    found = np.array([0, 0, 0, 1] + [0, 1, 1, 1] + [1] * 4, dtype=bool)
    s50, frac = weighting.snr50(snr, found, bins)
    assert np.allclose(frac, [0.25, 0.75, 1.0])
    assert s50 == pytest.approx(2.0)  # 0.25 at 1.5, 0.75 at 2.5: half way
    s50, _ = weighting.snr50(snr, np.zeros(12, bool), bins)
    assert np.isnan(s50)


def test_selection_counts_movers_and_unmatched():
    counts = np.array([30, 25, 19, 40, 22])
    matched = np.array([0, 2, 1, -1, -1])
    found, fp = weighting._selection(counts, matched, 22, 4)
    assert found.tolist() == [True, False, True, False] and fp == 2
    found, fp = weighting._selection(counts, matched, 100, 4)
    assert not found.any() and fp == 0


def test_likelihood_weights():
    w = synth.likelihood_weights(np.array([3.0, 5.0, 11.2, 20.0]), 4.0)
    assert w.dtype == np.uint8
    assert w.tolist() == [18, 50, 251, 255]  # round(2 s^2), capped


def test_faint_catalog_physics():
    wl = synth.make_faint(600, n_movers=100)
    mov = np.asarray(wl.is_mover) >= 0
    snr = np.asarray(wl.snr, dtype=np.float64)
    assert snr.min() >= 3.0  # every detection passed the SNR 3 cut
    # noise peaks follow the Gaussian tail above 3: mean about 3.28
    assert 3.2 < snr[~mov].mean() < 3.36
    # a mover's detected epochs grow with its true SNR
    mu = wl.truth["snr"]
    n_det = wl.truth["present"].sum(axis=1)
    assert np.corrcoef(mu, n_det)[0, 1] > 0.8
    assert wl.n_min == 0 and len(mu) == 100
