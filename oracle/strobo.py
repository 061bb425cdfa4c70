"""Oracle of stroboscopic resampling -- TEST INFRASTRUCTURE ONLY.

The comparison method of Sec. III.B and App. A, written out plainly in FP64:
the series, sampled at a rate O times higher than the resampled series
needs, is read at the sample nearest to each point of a uniform grid in the
resampled time tau (nearest-neighbour interpolation, i.e. convolution with
a rectangular kernel), and the Fourier sum of that tau-uniform series is
taken at the requested bins.  Only the tests and the benchmark use it.

Readings: the segment is its own reference (t_s = 0, u_s = 1); the tau grid
is tau_m = m / fs_O for every m with tau_m <= dtau(t_last); the time of a
grid point inverts Eq. (new_t), t = (3 / (8 beta)) (1 - (1 - tau/a)^{8/5}) with
a = 3 / (5 beta), evaluated with log1p/expm1; the nearest sample is
rint(t fs_O) (ties to even); the spectrum is S_k = (1/O) sum_m y_m
exp(-2 pi i f_k tau_m), which has the scale of the NUFFT sum over the
original samples.
"""
from __future__ import annotations

import math

import numpy as np

from . import beta as _beta


def tau_points(mc, f0, fs_o, n_samples):
    """Times t(tau_m) of the tau grid and its size M."""
    b = _beta(mc, f0) if mc > 0 else 0.0
    t_last = (n_samples - 1) / fs_o
    if b == 0.0:
        M = n_samples
        tau = np.arange(M) / fs_o
        return tau, tau.copy()
    a = 3.0 / (5.0 * b)
    dtau_max = a * (-math.expm1(0.625 * math.log1p(-(8.0 / 3.0) * b * t_last)))
    M = int(math.floor(dtau_max * fs_o)) + 1
    tau = np.arange(M) / fs_o
    return tau, time_of(tau, b)


def time_of(tau, b):
    """Eq. (new_t) solved for t (segment start as reference, u_s = 1):
    t = (3 / (8 beta)) (1 - (1 - tau / a)^{8/5}), a = 3 / (5 beta)."""
    tau = np.asarray(tau, dtype=np.float64)
    if b == 0.0:
        return tau.copy()
    a = 3.0 / (5.0 * b)
    return -np.expm1(1.6 * np.log1p(-tau / a)) * (3.0 / (8.0 * b))


def nearest(t, fs_o, n_samples):
    """Nearest-sample index of each time (-1 outside the series)."""
    n = np.rint(t * fs_o).astype(np.int64)
    return np.where((n >= 0) & (n < n_samples), n, -1)


def spectrum(x_o, fs_o, oversample, mc, f0, f_lo, df, K):
    """Stroboscopic spectrum S_k, k < K, of the oversampled segment x_o."""
    x_o = np.asarray(x_o)
    tau, t = tau_points(mc, f0, fs_o, len(x_o))
    n = nearest(t, fs_o, len(x_o))
    y = np.where(n >= 0, x_o[np.maximum(n, 0)], 0.0)
    out = np.empty(K, dtype=np.complex128)
    for k in range(K):
        f = f_lo + k * df
        ph = np.mod(f * tau, 1.0)
        out[k] = np.sum(y * np.exp(-2j * math.pi * ph)) / oversample
    return out


def tone_limit(amp_half, phi0, f_tone, M, fs_o, oversample, f_lo, df, K):
    """What S_k is for a series that is exactly (amp/2) exp(i (2 pi f_tone tau + phi0))
    on the tau grid (no interpolation error): a geometric series per bin."""
    out = np.empty(K, dtype=np.complex128)
    for k in range(K):
        th = 2.0 * math.pi * (f_tone - (f_lo + k * df)) / fs_o
        if abs(math.sin(0.5 * th)) < 1e-300:
            g = complex(M)
        else:
            # sum_{m<M} e^{i th m} = e^{i th (M-1)/2} sin(M th / 2) / sin(th / 2)
            g = np.exp(0.5j * th * (M - 1)) * math.sin(0.5 * M * th) / math.sin(0.5 * th)
        out[k] = amp_half * np.exp(1j * phi0) * g / oversample
    return out
