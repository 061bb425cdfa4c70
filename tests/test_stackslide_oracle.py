"""Pins of the stack-slide oracle (CPU): closed forms of Eq. (semicoherent_statistic)
on constructed power, the weight normalisation, and the track geometry
checked against where the (separately pinned) NUFFT oracle puts an
injected chirp's power."""
import math

import numpy as np
import pytest

import oracle
import synth
from oracle import stackslide as ss

BETAS, _ = synth.beta_bank(69)
GEOM = dict(t_coh=30.0, betas=BETAS, f_lo=40.0, df=1.0 / 30.0, f_start=40.0, f_max=60.0)


def _power(n_seg, value, n_bins=600):
    return np.full((len(BETAS), n_seg, n_bins), value)


def test_null_power_gives_zero():
    """P = mu in every cell: every track sums to exactly zero."""
    norm = 2.0 / 15360
    P = _power(12, 2.0 / norm)
    mcs = np.array([1e-3, 2e-2, 8e-2])
    out, cnt = ss.n_sigma(P, mcs, 2, norm=norm, **GEOM)
    assert np.all(cnt >= 0)
    assert np.allclose(out, 0.0, atol=1e-12)


def test_unit_excess_closed_form_and_bound():
    """P = mu + sigma: n_sigma = sum w = sum f^{4/3} / sqrt(sum f^{8/3}),
    at most sqrt(N) (Cauchy-Schwarz), and equal to sqrt(N) when the track
    frequency does not move (tiny Mc: equal weights)."""
    norm = 1.0
    n_seg = 10
    P = _power(n_seg, 4.0)
    for mc in (1e-6, 5e-2):
        out, cnt = ss.n_sigma(P, np.array([mc]), 1, norm=norm, **GEOM)
        for i0 in range(n_seg):
            N = cnt[0, i0]
            assert N >= 1
            assert out[0, i0] <= math.sqrt(N) + 1e-12
        if mc == 1e-6:
            assert np.allclose(out[0], np.sqrt(cnt[0]), rtol=1e-9)
        else:
            assert out[0, 0] < math.sqrt(cnt[0, 0]) - 1e-6


def test_weights_normalised_and_increasing():
    segs = ss.track(8e-2, 0.0, 200, **{k: GEOM[k] for k in ("t_coh", "betas", "f_lo", "df")},
                    n_bins=600, f_start=40.0, f_max=60.0)
    w = ss.weights(segs)
    assert len(segs) > 5
    assert abs(float(np.sum(w * w)) - 1.0) < 1e-12
    assert np.all(np.diff(w) > 0)                 # the chirp's amplitude grows with f
    f = np.array([s[3] for s in segs])
    assert np.all(np.diff(f) > 0) and f[0] == 40.0 and f[-1] <= 60.0


def test_track_ends_at_band_top_or_coalescence():
    # the Eq. (f) time to reach 60 Hz from 40 Hz: (3/8)(1/beta40 - 1/beta60)
    mc = 8e-2
    b40, b60 = oracle.beta(mc, 40.0), oracle.beta(mc, 60.0)
    t_sweep = 3.0 / 8.0 * (1.0 / b40 - 1.0 / b60)
    segs = ss.track(mc, 0.0, 400, 30.0, BETAS, 40.0, 1.0 / 30.0, 600, 40.0, 60.0)
    last = segs[-1][0] * 30.0
    assert last <= t_sweep < last + 30.0 + 1e-9


def test_injected_chirp_power_lies_on_its_track():
    """The NUFFT oracle's spectra of an injected 0PN chirp (Mc, t0) have their
    peak, in each on-track segment's nearest-beta template, at the track's
    bin; the statistic at the true (Mc, t0) beats its neighbours.  Spectra
    are computed for the on-track segments, beta templates k_i - 1 .. k_i + 1
    and bins j_i - 8 .. j_i + 8; other cells hold the noise mean."""
    mc, t0 = 1e-1, 45.0
    fs, t_coh = 256.0, 30.0
    w = synth.paper_bank(hours=0.3, fs=fs, t_coh=t_coh, inject=(mc, t0, 0.5, 0.3))
    n_seg, K = w.n_seg, int(w.n_bins[0])
    L = int(w.seg_len[0])
    norm = 2.0 / L
    segs = ss.track(mc, t0, n_seg, t_coh, BETAS, 40.0, 1.0 / t_coh, K, 40.0, 60.0)
    assert len(segs) >= 20
    P = np.full((len(BETAS), n_seg, K), 2.0 / norm)
    for (i, k, j, f) in segs:
        x = w.strain[w.seg_offset[i]:w.seg_offset[i] + L]
        lo, hi = max(0, j - 8), min(K, j + 9)
        for kk in range(max(0, k - 1), min(len(BETAS), k + 2)):
            X, ok = oracle.spectrum(x, fs, 0.0, w.mc[kk], 50.0, 40.0, 1.0 / t_coh, K,
                                    kidx=np.arange(lo, hi))
            assert ok
            P[kk, i, lo:hi] = np.abs(X) ** 2
        frac = (f - 40.0) * t_coh - math.floor((f - 40.0) * t_coh)
        peak = lo + int(np.argmax(P[k, i, lo:hi]))
        if abs(frac - 0.5) > 0.3:                    # bin edges sit at frac = 0.5
            assert peak == j, (i, k, j, peak)
        else:
            assert abs(peak - j) <= 1, (i, k, j, peak)
    # the nearest-beta templates hold more of the track's power than their neighbours
    on = sum(P[k, i, j] for (i, k, j, _) in segs)
    for dk in (-1, 1):
        off = sum(P[min(max(k + dk, 0), len(BETAS) - 1), i, j] for (i, k, j, _) in segs)
        assert on > off, (dk, on, off)
    S = 4
    i0 = int(math.ceil(t0 / t_coh))
    s_true = int(round((i0 * t_coh - t0) / t_coh * S))
    assert abs((i0 - s_true / S) * t_coh - t0) < 1e-9
    mcs = np.array([mc * 0.97, mc, mc * 1.03])
    cand = [(c, i0, s) for c in range(3) for s in range(S)]
    out, _ = ss.n_sigma(P, mcs, S, t_coh, BETAS, 40.0, 1.0 / t_coh, 40.0, 60.0, norm, tracks=cand)
    vals = {(c, s): out[c, i0 * S + s] for (c, _, s) in cand}
    best = max(vals, key=vals.get)
    assert best == (1, s_true), vals
    assert vals[(1, s_true)] > 20.0
