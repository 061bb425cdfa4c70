"""Pins of the oracle against what the paper and mathematics fix (CPU only).

Each test checks the oracle against something other than itself: numbers the
paper prints, closed forms, a library routine in a special case, identities
between different equations of the paper, and brute force at 50 digits.
"""
import json
import math
import os

import mpmath as mp
import numpy as np
import pytest

import oracle
import synth

GOLD = json.load(open(os.path.join(os.path.dirname(__file__), "golden", "paper_values.json")))


def _round_sig(x, n):
    return float(f"{x:.{n - 1}e}")


# ---------------------------------------------------------------- beta ----

def test_beta_range_matches_printed_bank_range():
    g = GOLD["beta_range"]
    bmin = oracle.beta(g["mc_lo"], g["f_lo"])
    bmax = oracle.beta(g["mc_hi"], g["f_hi"])
    assert _round_sig(bmin, g["sig_figs"]) == g["beta_min"]
    assert _round_sig(bmax, g["sig_figs"]) == g["beta_max"]
    # beta is monotone in both arguments, so the corners are the extremes
    grid = [oracle.beta(m, f) for m in np.geomspace(g["mc_lo"], g["mc_hi"], 7)
            for f in np.linspace(g["f_lo"], g["f_hi"], 5)]
    assert min(grid) == pytest.approx(bmin) and max(grid) == pytest.approx(bmax)


def test_chirp_durations_match_printed_values():
    g = GOLD["durations"]
    for c in g["cases"]:
        b = oracle.beta(c["mc"], g["f_from"])
        t = 3.0 / (8.0 * b) * (1.0 - (g["f_from"] / g["f_to"]) ** (8.0 / 3.0))  # Sec. II
        assert _round_sig(t / c["unit_s"], g["sig_figs"]) == c["value"]


def test_beta_scaling_exponents():
    # beta ~ Mc^{5/3} f0^{8/3}: doubling each argument scales by the power law
    b = oracle.beta(1e-2, 50.0)
    assert oracle.beta(2e-2, 50.0) / b == pytest.approx(2 ** (5 / 3), rel=1e-14)
    assert oracle.beta(1e-2, 100.0) / b == pytest.approx(2 ** (8 / 3), rel=1e-14)


# ----------------------------------------------------------------- tau ----

mp.mp.dps = 50


def _mp_tau(beta, t):
    u = 1 - mp.mpf(8) / 3 * beta * t
    return -mp.mpf(3) / 5 * u ** (mp.mpf(5) / 8) / beta


@pytest.mark.parametrize("mc,f0,ts", [(5e-4, 40.0, 0.0), (1e-2, 50.0, 0.0), (1e-2, 50.0, 1800.0),
                                      (1e-1, 60.0, 0.0), (3e-2, 45.0, 300.0)])
def test_dtau_matches_50_digit_evaluation(mc, f0, ts):
    fs, L = 256.0, 7680
    d = oracle.dtau(mc, f0, ts, fs, L)
    beta = mp.mpf(oracle.beta(mc, f0))
    j = np.array([0, 1, 2, 17, 1000, 4097, L - 1])
    ref = [float(_mp_tau(beta, mp.mpf(ts) + mp.mpf(int(i)) / fs) - _mp_tau(beta, mp.mpf(ts))) for i in j]
    assert np.max(np.abs(d[j] - np.array(ref))) < 1e-12


@pytest.mark.parametrize("mc,f0,ts", [(1e-1, 60.0, 0.0), (1e-2, 50.0, 900.0), (5e-4, 40.0, 0.0)])
def test_dtau_derivative_is_frequency_ratio(mc, f0, ts):
    # d tau / dt = f_0PN(t) / f0 with f_0PN from Eq. (f) -- a different equation
    fs, L = 4096.0, 4097
    d = oracle.dtau(mc, f0, ts, fs, L)
    b = oracle.beta(mc, f0)
    j = np.arange(1, L - 1, 97)
    t = ts + j / fs
    fd = (d[j + 1] - d[j - 1]) * fs / 2.0
    f_rat = (1.0 - (8.0 / 3.0) * b * t) ** (-3.0 / 8.0)
    # central difference error ~ h^2 tau''' / 6 is far below 1e-9 here
    assert np.max(np.abs(fd / f_rat - 1.0)) < 1e-9


@pytest.mark.parametrize("mc,f0,ts", [(1e-1, 60.0, 120.0), (1e-2, 50.0, 0.0), (1e-3, 41.0, 3000.0)])
def test_monochromatic_identity(mc, f0, ts):
    # Eq. (monochromatic): phi_0PN(t) = 2 pi f0 tau + phi0, with phi_0PN from Eq. (phi)
    fs, L = 256.0, 7680
    d = oracle.dtau(mc, f0, ts, fs, L)
    beta = mp.mpf(oracle.beta(mc, f0))

    def phi(t):
        return -6 * mp.pi / 5 * f0 * (1 - mp.mpf(8) / 3 * beta * t) ** (mp.mpf(5) / 8) / beta

    for j in (1, 333, 5000, L - 1):
        dphi = phi(mp.mpf(ts) + mp.mpf(j) / fs) - phi(mp.mpf(ts))
        assert abs(2 * math.pi * f0 * d[j] - float(dphi)) < 1e-9


def test_dtau_identity_limit():
    d = oracle.dtau(0.0, 50.0, 10.0, 256.0, 1000)
    assert np.array_equal(d, np.arange(1000) / 256.0)
    d = oracle.dtau(1e-12, 50.0, 0.0, 256.0, 1000)   # beta ~ 4e-22
    assert np.max(np.abs(d - np.arange(1000) / 256.0)) < 1e-12


# ------------------------------------------------------------ validity ----

@pytest.mark.parametrize("mc,f0", [(1e-1, 45.5), (3e-2, 52.5), (1e-1, 59.5)])
def test_validity_boundary_matches_duration_formula(mc, f0):
    # last valid segment ends before the chirp reaches f_max (Sec. II duration law)
    fs, T, fmax = 256.0, 30.0, 60.0
    b = oracle.beta(mc, f0)
    t_reach = 3.0 / (8.0 * b) * (1.0 - (f0 / fmax) ** (8.0 / 3.0))
    L = int(T * fs)
    for s in range(0, 400):
        ts = s * T
        t_last = ts + (L - 1) / fs
        v = oracle.valid(mc, f0, fmax, ts, fs, L)
        if abs(t_last - t_reach) > 1e-6:
            assert v == (t_last < t_reach)
    # with no frequency cut the boundary is coalescence, u = 0
    t_c = 3.0 / (8.0 * b)
    for s in range(0, 400):
        t_last = s * T + (L - 1) / fs
        if abs(t_last - t_c) > 1e-6:
            assert oracle.valid(mc, f0, 0.0, s * T, fs, L) == (t_last < t_c)


# ------------------------------------------------------------- spectra ----

def _rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


def _dirichlet(delta, N, fs):
    # sum_{j<N} exp(2 pi i delta j / fs)
    x = math.pi * delta / fs
    out = np.empty_like(delta, dtype=complex)
    small = np.abs(np.sin(x)) < 1e-300
    out[~small] = np.exp(1j * (N - 1) * x[~small]) * np.sin(N * x[~small]) / np.sin(x[~small])
    out[small] = N
    return out


@pytest.mark.parametrize("f_tone,phase", [(50.3, 0.0), (47.123, 1.1), (52.0, 0.4)])
def test_pure_tone_is_dirichlet_kernel(f_tone, phase):
    N, fs, K, df = 777, 256.0, 100, 0.05
    w = synth.pure_tone(L=N, fs=fs, f_tone=f_tone, phase=phase, f_lo=47.5, df=df, K=K)
    X, _, ok = oracle.spectra(w)
    f = 47.5 + np.arange(K) * df
    ref = 0.5 * (np.exp(1j * phase) * _dirichlet(f_tone - f, N, fs)
                 + np.exp(-1j * phase) * _dirichlet(-f_tone - f, N, fs))
    assert ok[0] and _rel(X, ref) < 1e-12


def test_identity_map_is_fft():
    N, fs = 512, 128.0
    x = np.random.default_rng(5).standard_normal(N)
    w = synth.pure_tone(L=N, fs=fs, f_lo=0.0, df=fs / N, K=N)
    w.strain = x
    X, _, _ = oracle.spectra(w)
    assert _rel(X, np.fft.fft(x)) < 1e-12


@pytest.mark.parametrize("mc,f0,ts", [(1e-2, 50.0, 0.0), (1e-1, 42.0, 0.0), (5e-3, 55.0, 0.0)])
def test_analytic_chirp_collapses_to_one_bin(mc, f0, ts):
    # resampling with the true template makes the chirp monochromatic (Sec. III.B)
    fs, T, A = 256.0, 30.0, 0.05
    L = int(T * fs)
    t = np.arange(L) / fs
    x = synth.injection(t, f0, mc, A, analytic=True)
    df = 1.0 / T
    X, ok = oracle.spectrum(x, fs, ts, mc, f0, f0 - 300 * df, df, 600)
    p = np.abs(X) ** 2
    assert ok and np.argmax(p) == 300
    assert abs(p[300] / (L * A / 2) ** 2 - 1.0) < 1e-9


def test_real_chirp_collapse_within_image_bound():
    w = synth.single_segment()
    L, A = 7680, w.meta["amp"]
    t = np.arange(L) / 256.0
    x = synth.injection(t, 50.0, 1e-2, A)                      # noise-free real chirp
    X, _ = oracle.spectrum(x, 256.0, 0.0, 1e-2, 50.0, 40.0, 1 / 30, 600)
    # the negative-frequency image I = sum_j (A/2) exp(-i(phi_j + 2 pi f0 dtau_j))
    xi = np.conj(synth.injection(t, 50.0, 1e-2, A, analytic=True))
    I, _ = oracle.spectrum(xi, 256.0, 0.0, 1e-2, 50.0, 50.0, 1.0, 1)
    main = L * A / 2
    rel = abs(abs(X[300]) ** 2 / main ** 2 - 1.0)
    assert rel <= 2 * abs(I[0]) / main + (abs(I[0]) / main) ** 2 + 1e-12
    assert np.argmax(np.abs(X)) == 300


def _mp_direct(x, fs, ts, beta, f_lo, df, K):
    out = []
    for k in range(K):
        fk = mp.mpf(f_lo) + k * mp.mpf(df)
        acc = mp.mpc(0)
        for j, xj in enumerate(x):
            if beta == 0:
                d = mp.mpf(j) / fs
            else:
                d = _mp_tau(beta, mp.mpf(ts) + mp.mpf(j) / fs) - _mp_tau(beta, mp.mpf(ts))
            acc += mp.mpc(xj) * mp.exp(-2j * mp.pi * fk * d)
        out.append(complex(acc))
    return np.array(out)


@pytest.mark.parametrize("seed,L,K,mc,ts,cplx", [
    (0, 16, 8, 1e-2, 0.0, False), (1, 33, 40, 1e-1, 60.0, True), (2, 64, 12, 5e-4, 0.0, False),
    (3, 5, 9, 3e-2, 30.0, True), (4, 48, 48, 0.0, 0.0, False), (5, 1, 3, 1e-2, 0.0, False)])
def test_brute_force_50_digits(seed, L, K, mc, ts, cplx):
    mp.mp.dps = 50
    w = synth.random_small(seed, L, K, mc, f0=50.0, fs=64.0, t_start=ts, complex_strain=cplx)
    X, _, ok = oracle.spectra(w)
    beta = mp.mpf(oracle.beta(mc, 50.0)) if mc else 0
    ref = _mp_direct(w.strain, 64.0, ts, beta, w.f_lo[0], w.df[0], K)
    assert ok[0] and _rel(X, ref) < 1e-13


def test_real_input_conjugate_symmetry():
    L, fs, mc, f0 = 300, 64.0, 2e-2, 50.0
    x = np.random.default_rng(9).standard_normal(L)
    df = 0.1
    Xp, _ = oracle.spectrum(x, fs, 0.0, mc, f0, 10.0, df, 20)
    Xm, _ = oracle.spectrum(x, fs, 0.0, mc, f0, -10.0 - 19 * df, df, 20)
    assert _rel(Xm[::-1], np.conj(Xp)) < 1e-13


def test_linearity():
    L, fs = 200, 64.0
    rng = np.random.default_rng(11)
    x, y = rng.standard_normal(L), rng.standard_normal(L)
    a, b = 0.7, -2.3
    args = (fs, 5.0, 3e-2, 45.0, 40.0, 0.1, 30)
    X, _ = oracle.spectrum(x, *args)
    Y, _ = oracle.spectrum(y, *args)
    Z, _ = oracle.spectrum(a * x + b * y, *args)
    assert _rel(Z, a * X + b * Y) < 1e-13


def test_noise_normalised_power_is_chi2_two_dof():
    # P = 4|x~|^2/(T S) with x~ = X/fs and S = 2 sigma^2/fs gives 2|X|^2/(L sigma^2)
    g = GOLD["noise_power"]
    w = synth.semicoherent(hours=0.25, n_mc=2, n_sub=20, seed=4, inject=False)
    X, off, ok = oracle.spectra(w, inst_idx=np.arange(0, w.n_inst, 3))
    L = 7680
    P = 2.0 * np.abs(X[np.repeat(ok.astype(bool), 30)]) ** 2 / L
    assert P.size > 3000
    assert abs(P.mean() - g["mean"]) < 0.1 and abs(P.std() - g["std"]) < 0.15


# --------------------------------------------------------- segment sum ----

def test_segment_sum_is_sum_of_valid_powers_and_order_free():
    w = synth.semicoherent(hours=0.1, n_mc=3, n_sub=2, seed=6, snr=10.0)
    w.seg_len = np.full(w.n_seg, 700, np.int64)                    # shorter segments, quicker
    stat, off, used = oracle.semicoherent(w)
    X, xoff, ok = oracle.spectra(w)
    P = np.abs(X) ** 2
    for m in range(w.n_tmpl):
        K = w.n_bins[m]
        acc = np.zeros(K)
        for s in range(w.n_seg):
            i = m * w.n_seg + s
            if ok[i]:
                acc += P[xoff[i]:xoff[i] + K]
        assert np.allclose(stat[off[m]:off[m + 1]], acc, rtol=1e-13, atol=0)
        assert used[m] == ok[m * w.n_seg:(m + 1) * w.n_seg].sum()
    # reversing the segment order (moving the data with it) leaves the sum unchanged
    wr = synth.Workload(**{**w.__dict__})
    wr.seg_offset = w.seg_offset[::-1].copy(); wr.seg_t = w.seg_t[::-1].copy()
    stat_r, _, used_r = oracle.semicoherent(wr)
    assert np.allclose(stat_r, stat, rtol=1e-13) and np.array_equal(used_r, used)
    # weights enter linearly
    wts = np.linspace(0.5, 1.5, w.n_seg)
    stat_w, _, _ = oracle.semicoherent(w, seg_weight=wts)
    m = 0
    acc = sum(wts[s] * P[xoff[m * w.n_seg + s]:xoff[m * w.n_seg + s] + w.n_bins[m]]
              for s in range(w.n_seg) if ok[m * w.n_seg + s])
    assert np.allclose(stat_w[off[0]:off[1]], acc, rtol=1e-13)
