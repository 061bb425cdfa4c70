"""Seeded synthetic inputs shared by the oracle tests and the GPU path.

This module only draws random numbers and builds strain arrays and workload
descriptions (segments, templates, instances).  It holds none of the
resampling / NUFFT / power / segment-sum arithmetic.  The injected signal is
the paper's Newtonian (0PN) inspiral: frequency law Eq. (f) and phase law
Eq. (phi) of Sec. III.A, with the chirp-mass parameter beta of Eq. (beta) in
Sec. II.  The phase offset phi0 is taken to be the phase at the reference time
t0, i.e. the injected phase is phi_0PN(t) - phi_0PN(t0) + phi0.

Random draw order (numpy PCG64 ``default_rng(seed)``): the noise first, then
the injection parameters, in the order documented per workload.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

# GM_sun / c^3 in seconds, from the IAU 2015 nominal solar mass parameter
# GM_sun = 1.3271244e20 m^3 s^-2 and the exact speed of light.
GM_SUN = 1.3271244e20
C_LIGHT = 299792458.0
T_SUN = GM_SUN / C_LIGHT ** 3

MC_MIN, MC_MAX = 5e-4, 1e-1      # chirp-mass range of the search (abstract, Sec. III.A)
BAND_LO, BAND_HI = 40.0, 60.0    # analysed band (Sec. III.C / IV)


def chirp_beta(mc_msun, f0):
    """beta(f0, Mc) of Eq. (beta), in s^-1 (numpy float64)."""
    mc = np.asarray(mc_msun, dtype=np.float64)
    f = np.asarray(f0, dtype=np.float64)
    return (96.0 / 5.0) * math.pi ** (8.0 / 3.0) * (T_SUN * mc) ** (5.0 / 3.0) * f ** (8.0 / 3.0)


def chirp_phase(t, f0, mc_msun, t0=0.0, phi0=0.0):
    """Injected 0PN phase, Eq. (phi) relative to its value at t0, plus phi0.

    Evaluated as (6 pi/5)(f0/beta)(1 - u^{5/8}) with u = 1 - (8/3) beta (t - t0),
    written with log1p/expm1 so that thousands of cycles keep ~1e-12 rad
    accuracy.  Returns NaN where u <= 0 (past coalescence).
    """
    t = np.asarray(t, dtype=np.float64)
    b = float(chirp_beta(mc_msun, f0))
    if b == 0.0:
        return 2.0 * math.pi * f0 * (t - t0) + phi0
    y = (8.0 / 3.0) * b * (t - t0)
    with np.errstate(invalid="ignore", divide="ignore"):
        one_minus = -np.expm1(0.625 * np.log1p(-y))
    return (6.0 * math.pi / 5.0) * (f0 / b) * one_minus + phi0


def chirp_frequency(t, f0, mc_msun, t0=0.0):
    """Instantaneous 0PN frequency, Eq. (f); NaN past coalescence."""
    t = np.asarray(t, dtype=np.float64)
    b = float(chirp_beta(mc_msun, f0))
    u = 1.0 - (8.0 / 3.0) * b * (t - t0)
    with np.errstate(invalid="ignore", divide="ignore"):
        return np.where(u > 0, f0 * np.abs(u) ** (-0.375), np.nan)


def injection(t, f0, mc_msun, amp, t0=0.0, phi0=0.0, analytic=False, f_stop=None):
    """A constant-amplitude 0PN chirp sampled at times t.

    Real form amp*cos(Phi); analytic form (amp/2)*exp(i*Phi).  Samples past
    coalescence, or where the chirp frequency exceeds f_stop, are zero.
    """
    ph = chirp_phase(t, f0, mc_msun, t0, phi0)
    f = chirp_frequency(t, f0, mc_msun, t0)
    on = np.isfinite(ph) & np.isfinite(f)
    if f_stop is not None:
        on &= f <= f_stop
    ph = np.where(on, ph, 0.0)
    if analytic:
        return np.where(on, 0.5 * amp * np.exp(1j * ph), 0.0)
    return np.where(on, amp * np.cos(ph), 0.0)


# --------------------------------------------------------------------------
# Workload descriptions
# --------------------------------------------------------------------------

@dataclass
class Workload:
    """Segments x templates (x optional explicit instances) over one strain."""
    name: str
    strain: np.ndarray                     # float64 (real) or complex128
    seg_offset: np.ndarray                 # int64 [S]
    seg_len: np.ndarray                    # int64 [S]
    seg_fs: np.ndarray                     # float64 [S]
    seg_t: np.ndarray                      # float64 [S], start time relative to t0
    mc: np.ndarray                         # float64 [M]
    f0: np.ndarray                         # float64 [M]
    f_lo: np.ndarray                       # float64 [M]
    df: np.ndarray                         # float64 [M] (<=0: 1/T of the segment)
    n_bins: np.ndarray                     # int32 [M]
    f_max: np.ndarray                      # float64 [M] (<=0: no frequency cut)
    inst_seg: np.ndarray | None = None     # int32 [I]; None: full product, template-major
    inst_tmpl: np.ndarray | None = None
    inst_tol: np.ndarray | None = None     # float64 [I]; None: the plan tolerance
    tol: float = 1e-6
    meta: dict = field(default_factory=dict)

    @property
    def n_seg(self):
        return len(self.seg_offset)

    @property
    def n_tmpl(self):
        return len(self.mc)

    def instances(self):
        """(seg, tmpl) int32 arrays; the full product is template-major."""
        if self.inst_seg is not None:
            return self.inst_seg.astype(np.int32), self.inst_tmpl.astype(np.int32)
        s = np.tile(np.arange(self.n_seg, dtype=np.int32), self.n_tmpl)
        m = np.repeat(np.arange(self.n_tmpl, dtype=np.int32), self.n_seg)
        return s, m

    @property
    def n_inst(self):
        return len(self.inst_seg) if self.inst_seg is not None else self.n_seg * self.n_tmpl

    def bins_per_instance(self):
        s, m = self.instances()
        return self.n_bins[m].astype(np.int64)

    def bin_offsets(self):
        k = self.bins_per_instance()
        off = np.zeros(len(k) + 1, dtype=np.int64)
        np.cumsum(k, out=off[1:])
        return off

    def subset(self, inst_idx):
        """Explicit-instance copy restricted to the given instance indices."""
        s, m = self.instances()
        idx = np.asarray(inst_idx, dtype=np.int64)
        tol = None if self.inst_tol is None else self.inst_tol[idx]
        w = Workload(**{**self.__dict__, "inst_seg": s[idx].copy(), "inst_tmpl": m[idx].copy(),
                        "inst_tol": tol, "meta": dict(self.meta)})
        return w

    def as_float32_strain(self):
        """Copy whose strain is rounded to float32 values (kept as float64)."""
        w = Workload(**{**self.__dict__, "meta": dict(self.meta)})
        if np.iscomplexobj(self.strain):
            w.strain = self.strain.astype(np.complex64).astype(np.complex128)
        else:
            w.strain = self.strain.astype(np.float32).astype(np.float64)
        return w


def log_spaced_mc(m):
    """Inclusive log spacing of the chirp-mass range, Mc_m = Mc_min (Mc_max/Mc_min)^{m/(M-1)}."""
    if m == 1:
        return np.array([MC_MIN])
    return MC_MIN * (MC_MAX / MC_MIN) ** (np.arange(m) / (m - 1.0))


def _subband_templates(n_mc, n_sub=20, t_coh=30.0, f_max=BAND_HI):
    mcs = log_spaced_mc(n_mc)
    mc = np.repeat(mcs, n_sub)
    b = np.tile(np.arange(n_sub), n_mc).astype(np.float64)
    f_lo = BAND_LO + b
    f0 = f_lo + 0.5
    df = np.full(mc.shape, 1.0 / t_coh)
    K = np.full(mc.shape, int(round(1.0 / (1.0 / t_coh))), dtype=np.int32)
    return mc, f0, f_lo, df, K, np.full(mc.shape, f_max)


def _segments(n_seg, L, fs):
    off = np.arange(n_seg, dtype=np.int64) * L
    return (off, np.full(n_seg, L, np.int64), np.full(n_seg, float(fs)),
            np.arange(n_seg, dtype=np.float64) * (L / fs))


def single_segment(seed=0, analytic=False):
    """30 s at 256 Hz of N(0,1) noise plus a 0PN chirp (Mc=1e-2, 50 Hz at the start,
    amplitude 0.05, phi0=0); one template at the true chirp, 600 bins of 1/30 Hz over
    40-60 Hz; tolerance 1e-9 in double precision."""
    fs, T = 256.0, 30.0
    L = int(round(T * fs))
    rng = np.random.default_rng(seed)
    noise = rng.standard_normal(L)
    t = np.arange(L) / fs
    x = noise + injection(t, 50.0, 1e-2, 0.05, analytic=analytic)
    if analytic:
        x = x.astype(np.complex128)
    return Workload(
        name="single_segment_30s_fp64", strain=x,
        seg_offset=np.array([0], np.int64), seg_len=np.array([L], np.int64),
        seg_fs=np.array([fs]), seg_t=np.array([0.0]),
        mc=np.array([1e-2]), f0=np.array([50.0]), f_lo=np.array([40.0]),
        df=np.array([1.0 / 30.0]), n_bins=np.array([600], np.int32), f_max=np.array([BAND_HI]),
        tol=1e-9, meta={"amp": 0.05, "mc": 1e-2, "f_inj": 50.0})


def semicoherent(hours=1.0, n_mc=64, n_sub=20, seed=1, snr=20.0, fs=256.0, t_coh=30.0,
                 tol=1e-6, inject=True):
    """hours of N(0,1) noise at fs split into t_coh segments, plus one 0PN chirp with
    Mc log-uniform over the search range, start frequency uniform in 40-60 Hz at t0
    (the observation start) and phi0 uniform; amplitude set for optimal SNR ``snr``
    (white noise: rho^2 = sum h_j^2).  Templates: n_mc log-spaced chirp masses x n_sub
    sub-bands of 1 Hz over 40-60 Hz with f0 at the sub-band centre.
    Draw order: noise, then log10(Mc), f, phi0."""
    L = int(round(t_coh * fs))
    n_seg = int(round(hours * 3600.0 / t_coh))
    N = n_seg * L
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(N)
    meta = {}
    if inject:
        lmc = rng.uniform(math.log10(MC_MIN), math.log10(MC_MAX))
        f_inj = rng.uniform(BAND_LO, BAND_HI)
        phi0 = rng.uniform(0.0, 2.0 * math.pi)
        mc_inj = 10.0 ** lmc
        t = np.arange(N) / fs
        h = injection(t, f_inj, mc_inj, 1.0, phi0=phi0, f_stop=0.45 * fs)
        e = float(np.sum(h * h))
        amp = snr / math.sqrt(e) if e > 0 else 0.0
        x = x + amp * h
        meta = {"mc": mc_inj, "f_inj": f_inj, "phi0": phi0, "amp": amp, "snr": snr}
    off, ln, fsa, ts = _segments(n_seg, L, fs)
    mc, f0, f_lo, df, K, fmax = _subband_templates(n_mc, n_sub, t_coh)
    return Workload(name=f"semicoherent_{hours:g}h_{n_mc}x{n_sub}", strain=x,
                    seg_offset=off, seg_len=ln, seg_fs=fsa, seg_t=ts,
                    mc=mc, f0=f0, f_lo=f_lo, df=df, n_bins=K, f_max=fmax, tol=tol, meta=meta)


def ragged_batch(n_inst=512, seed=2):
    """n_inst independent instances, each one segment of T in {10,30,60} s at fs in
    {256,512,1024} Hz with tolerance in {1e-3,1e-6,1e-9}, uniform over the 27
    combinations; N(0,1) noise plus a 0PN chirp (Mc log-uniform, f uniform 40-60 Hz,
    phi0 uniform, amplitude 0.05); one template at the true chirp analysing the full
    40-60 Hz band with 1/T bins.  Draw order per instance: combination, noise,
    log10(Mc), f, phi0."""
    Ts, fss, tols = (10.0, 30.0, 60.0), (256.0, 512.0, 1024.0), (1e-3, 1e-6, 1e-9)
    rng = np.random.default_rng(seed)
    chunks, off, ln, fsv, tv, mc, f0, tol = [], [], [], [], [], [], [], []
    pos = 0
    for _ in range(n_inst):
        c = int(rng.integers(27))
        T, fs, tl = Ts[c // 9], fss[(c // 3) % 3], tols[c % 3]
        L = int(round(T * fs))
        noise = rng.standard_normal(L)
        m = 10.0 ** rng.uniform(math.log10(MC_MIN), math.log10(MC_MAX))
        f = rng.uniform(BAND_LO, BAND_HI)
        ph = rng.uniform(0.0, 2.0 * math.pi)
        t = np.arange(L) / fs
        chunks.append(noise + injection(t, f, m, 0.05, phi0=ph, f_stop=0.45 * fs))
        off.append(pos); ln.append(L); fsv.append(fs); tv.append(0.0)
        mc.append(m); f0.append(f); tol.append(tl)
        pos += L
    n = len(off)
    K = np.array([int(round((BAND_HI - BAND_LO) * L / fs)) for L, fs in zip(ln, fsv)], np.int32)
    return Workload(
        name=f"ragged_{n_inst}", strain=np.concatenate(chunks),
        seg_offset=np.array(off, np.int64), seg_len=np.array(ln, np.int64),
        seg_fs=np.array(fsv), seg_t=np.array(tv),
        mc=np.array(mc), f0=np.array(f0), f_lo=np.full(n, BAND_LO), df=np.zeros(n),
        n_bins=K, f_max=np.zeros(n),
        inst_seg=np.arange(n, dtype=np.int32), inst_tmpl=np.arange(n, dtype=np.int32),
        inst_tol=np.array(tol), tol=1e-6, meta={})


def pure_tone(L=256, fs=256.0, f_tone=50.3, amp=1.0, f_lo=40.0, df=None, K=64, phase=0.0,
              analytic=False):
    """Identity resampling (Mc = 0): a pure tone sampled uniformly, one segment."""
    t = np.arange(L) / fs
    x = amp * (np.exp(1j * (2 * math.pi * f_tone * t + phase)) if analytic
               else np.cos(2 * math.pi * f_tone * t + phase))
    df = fs / L if df is None else df
    return Workload(
        name="pure_tone", strain=x,
        seg_offset=np.array([0], np.int64), seg_len=np.array([L], np.int64),
        seg_fs=np.array([fs]), seg_t=np.array([0.0]),
        mc=np.array([0.0]), f0=np.array([f_tone]), f_lo=np.array([f_lo]),
        df=np.array([df]), n_bins=np.array([K], np.int32), f_max=np.array([0.0]), tol=1e-9)


def random_small(seed, L, K, mc, f0=50.0, fs=64.0, f_lo=None, df=None, t_start=0.0,
                 complex_strain=False):
    """One short random segment with one template (brute-force sized cases)."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(L)
    if complex_strain:
        x = x + 1j * rng.standard_normal(L)
    df = (fs / L) if df is None else df
    f_lo = (f0 - (K // 2) * df) if f_lo is None else f_lo
    return Workload(
        name="random_small", strain=x,
        seg_offset=np.array([0], np.int64), seg_len=np.array([L], np.int64),
        seg_fs=np.array([fs]), seg_t=np.array([t_start]),
        mc=np.array([mc]), f0=np.array([f0]), f_lo=np.array([f_lo]), df=np.array([df]),
        n_bins=np.array([K], np.int32), f_max=np.array([0.0]), tol=1e-9)


# --------------------------------------------------------------------------
# Learned-proposal inputs
# --------------------------------------------------------------------------

MLP_SHAPES = [("W1", (256, 64)), ("b1", (256,)), ("W2", (256, 256)), ("b2", (256,)),
              ("w3", (256,)), ("b3", (1,))]


def mlp_init_params(seed):
    """He-uniform initial weights and zero biases of the 64-256-256-1 network,
    flattened as W1[256][64], b1, W2[256][256], b2, w3[256], b3 (float32)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in MLP_SHAPES:
        if name.startswith("b"):
            parts.append(np.zeros(shape))
        else:
            fan_in = shape[-1] if len(shape) == 2 else 256
            lim = math.sqrt(6.0 / fan_in)
            parts.append(rng.uniform(-lim, lim, size=shape))
    return np.concatenate([q.ravel() for q in parts]).astype(np.float32)


def beta_bank(n_beta=69, beta_lo=3e-8, beta_hi=7e-4, f0=50.0):
    """Chirp masses of a bank uniform in beta (Sec. III.A: 69 templates over
    3e-8 <= beta <= 7e-4), expressed at the template frequency f0:
    Mc = (beta / ((96/5) pi^{8/3} T_sun^{5/3} f0^{8/3}))^{3/5}."""
    betas = np.linspace(beta_lo, beta_hi, n_beta)
    c = (96.0 / 5.0) * math.pi ** (8.0 / 3.0) * T_SUN ** (5.0 / 3.0) * f0 ** (8.0 / 3.0)
    return betas, (betas / c) ** 0.6


def paper_bank(hours=1.0, seed=5, fs=512.0, t_coh=30.0, n_beta=69, inject=None):
    """The paper's coherent workload (Sec. III.A, VI): 30 s segments at 512 Hz,
    each resampled with every one of 69 beta templates (uniform over
    [3e-8, 7e-4], beta(f0 = 50 Hz, Mc)) referenced at the segment's own start,
    and transformed onto the full 40-60 Hz band in bins of 1/T_coh (600 at
    30 s).  N(0,1) noise; inject = (Mc, t0, amplitude, phi0) adds a 0PN chirp
    that passes 40 Hz at time t0 (stops at 0.45 fs).  Every segment has
    seg_t = 0: its own start is the resampling reference."""
    L = int(round(t_coh * fs))
    n_seg = int(round(hours * 3600.0 / t_coh))
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(n_seg * L)
    if inject is not None:
        mc_i, t0_i, amp, ph = inject
        t = np.arange(n_seg * L) / fs
        x = x + injection(t, BAND_LO, mc_i, amp, t0=t0_i, phi0=ph, f_stop=0.45 * fs)
    off, ln, fsa, _ = _segments(n_seg, L, fs)
    _, mc = beta_bank(n_beta)
    m = len(mc)
    K = int(round((BAND_HI - BAND_LO) * t_coh))
    return Workload(name=f"paper_beta_bank_{hours:g}h_{n_beta}beta_{fs:g}Hz", strain=x,
                    seg_offset=off, seg_len=ln, seg_fs=fsa, seg_t=np.zeros(n_seg),
                    mc=mc, f0=np.full(m, 50.0), f_lo=np.full(m, BAND_LO), df=np.full(m, 1.0 / t_coh),
                    n_bins=np.full(m, K, np.int32), f_max=np.zeros(m), tol=1e-6,
                    meta={"t_coh": t_coh, "inject": inject})


def noise_power(n_beta, n_seg, n_bins, L, seed=0, excess=None):
    """Stand-in stored spectra for the stack-slide: |X|^2 of white N(0,1) noise
    over L samples (L/2 times a chi^2_2 variate), float32 [n_beta][n_seg][n_bins].
    excess: optional list of (k, i, j, value) cells set to value."""
    rng = np.random.default_rng(seed)
    p = (0.5 * L) * rng.chisquare(2.0, size=(n_beta, n_seg, n_bins))
    if excess:
        for (k, i, j, v) in excess:
            p[k, i, j] = v
    return p.astype(np.float32)
