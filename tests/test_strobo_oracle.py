"""Pins of the stroboscopic-resampling oracle (CPU): the identity map is the
plain DFT (numpy's FFT), the inverse time map undoes the NUFFT oracle's
Eq. (new_t), and an analytic chirp converges to its tau-uniform tone at the
first-order rate of nearest-neighbour interpolation."""
import math

import numpy as np

import oracle
import synth
from oracle import strobo


def test_identity_map_with_no_oversampling_is_the_dft():
    rng = np.random.default_rng(0)
    L, fs = 512, 64.0
    x = rng.standard_normal(L) + 1j * rng.standard_normal(L)
    S = strobo.spectrum(x, fs, 1, 0.0, 20.0, 10.0, fs / L, 40)
    ref = np.fft.fft(x)[80:120]
    assert np.allclose(S, ref, rtol=1e-11, atol=1e-9)


def test_inverse_time_map_undoes_eq_new_t():
    mc, f0, fs, L = 3e-2, 20.0, 512.0, 4096
    dt = oracle.dtau(mc, f0, 0.0, fs, L)          # the NUFFT oracle's tau differences
    b = oracle.beta(mc, f0)
    t = strobo.time_of(dt, b)
    assert np.allclose(t, np.arange(L) / fs, rtol=0, atol=1e-11)
    assert np.array_equal(strobo.nearest(t, fs, L), np.arange(L))


def test_analytic_chirp_converges_first_order():
    """Nearest-neighbour timing errors of an analytic chirp shrink as 1/O once
    the chirp's drift away from uniform time spans several samples."""
    mc, f0, amp, phi0 = 1e-1, 20.0, 1.0, 0.4
    fs, T = 128.0, 16.0
    f_lo, df, K = 18.0, 1.0 / T, 64
    errs = []
    for O in (4, 8, 16, 32, 64):
        fs_o = fs * O
        n = int(round(T * fs_o))
        x = 0.5 * amp * np.exp(1j * synth.chirp_phase(np.arange(n) / fs_o, f0, mc, 0.0, phi0))
        S = strobo.spectrum(x, fs_o, O, mc, f0, f_lo, df, K)
        tau, _ = strobo.tau_points(mc, f0, fs_o, n)
        ref = strobo.tone_limit(0.5 * amp, phi0, f0, len(tau), fs_o, O, f_lo, df, K)
        errs.append(np.linalg.norm(S - ref) / np.linalg.norm(ref))
    ratios = [errs[q] / errs[q + 1] for q in range(len(errs) - 1)]
    assert errs[0] < 0.1 and errs[-1] < 5e-3, errs
    assert all(1.6 < r < 3.2 for r in ratios), (errs, ratios)
