"""Oracle of the weighted stack-slide along 0PN tracks -- TEST INFRASTRUCTURE ONLY.

A plain FP64 evaluation, one track at a time, of the semicoherent statistic
of Sec. III.C, Eq. (semicoherent_statistic), over stored per-segment power
spectra.  Only the tests and the benchmark's CPU leg may use it.

Readings (listed with the others in the design notes):
  * segment i is resampled with its beta templates referenced at its own
    start t_i = i T_coh, so the stored power of segment i, beta template k,
    bin j is |X|^2 at f_j = f_lo + j df;
  * the semicoherent template theta = (Mc, t0) passes f_start (the band's
    lower edge, Sec. III.C) at t0; segment i lies on the track when
    t_i >= t0 and its Eq. (f) frequency f_i = f_start u_i^{-3/8},
    u_i = 1 - (8/3) beta(f_start, Mc) (t_i - t0), is defined (u_i > 0), at
    most f_max, and rounds to a bin of the band;
  * its beta template is the bank entry nearest beta(f_i, Mc) = beta_start / u_i
    (the lower index on a tie), its bin round(f_i - f_lo)/df (halves up);
  * weights (Eq. (weights)) for white noise and no window: A_i^2 of the 0PN
    amplitude grows as f_i^{4/3}, S and Gamma are constant, so
    w_i = f_i^{4/3} / sqrt(sum over the track of f^{8/3}) (sum of w^2 = 1);
  * P = norm |X|^2 is Eq. (normalized_power) (norm = 2/(L sigma^2)), and
    n_sigma = sum_i w_i (P_i - mu) / sigma with mu = sigma = 2 for Gaussian
    noise (Sec. III.C); a track with no segment has n_sigma = 0.
"""
from __future__ import annotations

import math

import numpy as np

from . import beta as _beta


def _segment(b0, dt, betas, f_lo, df, n_bins, f_start, f_max):
    """(k, j, f) of a segment dt after t0, or None once the track has ended."""
    u = 1.0 - (8.0 / 3.0) * b0 * dt
    if not u > 0.0:
        return None
    f = f_start * u ** (-3.0 / 8.0)
    if f > f_max:
        return None
    j = math.floor((f - f_lo) / df + 0.5)
    if j < 0 or j >= n_bins:
        return None
    k = int(np.argmin(np.abs(betas - b0 / u)))       # first minimum: the lower index on a tie
    return k, j, f


def track(mc, t0, n_seg, t_coh, betas, f_lo, df, n_bins, f_start, f_max):
    """Segments of one track: list of (i, k, j, f_i) in segment order."""
    b0 = _beta(mc, f_start)
    out = []
    betas = np.asarray(betas, dtype=np.float64)
    for i in range(n_seg):
        ti = i * t_coh
        if ti < t0:
            continue
        r = _segment(b0, ti - t0, betas, f_lo, df, n_bins, f_start, f_max)
        if r is None:
            break
        out.append((i,) + r)
    return out


def track_grid(mc, i0, s, t0_steps, n_seg, t_coh, betas, f_lo, df, n_bins, f_start, f_max):
    """The track with t0 = (i0 - s / S) t_coh, with segment i0 + m at
    t_i - t0 = (m + s / S) t_coh (the grid form of the same times)."""
    b0 = _beta(mc, f_start)
    betas = np.asarray(betas, dtype=np.float64)
    out = []
    for m in range(n_seg - i0):
        r = _segment(b0, (m + s / t0_steps) * t_coh, betas, f_lo, df, n_bins, f_start, f_max)
        if r is None:
            break
        out.append((i0 + m,) + r)
    return out


def weights(segs):
    """Eq. (weights) for white noise: w_i proportional to f_i^{4/3}, sum w^2 = 1."""
    if not segs:
        return np.zeros(0)
    a = np.array([f ** (4.0 / 3.0) for (_, _, _, f) in segs])
    return a / math.sqrt(float(np.sum(a * a)))


def n_sigma_one(power_kij, segs, norm, mu=2.0, sigma=2.0):
    """Eq. (semicoherent_statistic) of one track; power_kij[k][i][j] holds |X|^2."""
    w = weights(segs)
    s = 0.0
    for q, (i, k, j, _) in enumerate(segs):
        s += w[q] * (norm * float(power_kij[k, i, j]) - mu) / sigma
    return s


def n_sigma(power_kij, mcs, t0_steps, t_coh, betas, f_lo, df, f_start, f_max, norm, mu=2.0, sigma=2.0,
            tracks=None):
    """n_sigma and segment counts of the tracks (Mc index c, t0 = (i0 - s / S) T_coh)
    for S = t0_steps, stored at [c][i0 * S + s].  tracks: optional list of
    (c, i0, s) to evaluate (the rest stay NaN)."""
    P = np.asarray(power_kij, dtype=np.float64)
    n_beta, n_seg, n_bins = P.shape
    out = np.full((len(mcs), n_seg * t0_steps), np.nan)
    cnt = np.full((len(mcs), n_seg * t0_steps), -1, dtype=np.int64)
    if tracks is None:
        tracks = [(c, i0, s) for c in range(len(mcs)) for i0 in range(n_seg) for s in range(t0_steps)]
    for (c, i0, s) in tracks:
        segs = track_grid(mcs[c], i0, s, t0_steps, n_seg, t_coh, betas, f_lo, df, n_bins, f_start, f_max)
        out[c, i0 * t0_steps + s] = n_sigma_one(P, segs, norm, mu, sigma)
        cnt[c, i0 * t0_steps + s] = len(segs)
    return out, cnt
