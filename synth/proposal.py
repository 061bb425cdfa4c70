"""Seeded inputs of the learned-proposal workload.

The search layout (segments, sub-bands), the coarse and fine chirp-mass
grids, the region an injection belongs to, and injection draws: numpy for
single draws shared with the oracle, torch on the device for the large
training and judging sets.  Like the rest of ``synth`` this module only
describes workloads and draws random inputs; it holds none of the
resampling, NUFFT, power, sum or network arithmetic.

Region and label convention: a region is (coarse cell m, sub-band b); an
injection (Mc, f at t0) belongs to the sub-band b holding f and to the cell
containing Mc* = Mc (f / f0_b)^{8/5}, f0_b the sub-band centre, because
beta(f0_b, Mc*) = beta(f, Mc) (Eq. (beta)): the template with that beta at
f0_b resamples the chirp exactly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import MC_MAX, MC_MIN, Workload, chirp_beta, injection


@dataclass(frozen=True)
class Layout:
    """n_seg segments of t_coh seconds at fs, searched in n_sub sub-bands of
    1 Hz from band_lo (f0 at each sub-band's centre, bins of 1/t_coh)."""
    n_seg: int = 120
    t_coh: float = 30.0
    fs: float = 256.0
    n_sub: int = 20
    band_lo: float = 40.0

    @property
    def L(self):
        return int(round(self.t_coh * self.fs))

    @property
    def K(self):
        return int(round(self.t_coh))          # 1 Hz of 1/t_coh bins

    @property
    def samples(self):
        return self.n_seg * self.L

    @property
    def norm(self):
        """1 / (L sigma^2) for unit-variance noise: |X|^2 norm has unit mean."""
        return 1.0 / self.L

    @property
    def band_hi(self):
        return self.band_lo + self.n_sub


@dataclass(frozen=True)
class Grid:
    """Coarse chirp-mass grid: n_mc cell centres log-spaced over [MC_MIN, MC_MAX];
    cell m spans half a log step either side of its centre (clipped to the range)."""
    n_mc: int

    @property
    def log_step(self):
        return math.log(MC_MAX / MC_MIN) / (self.n_mc - 1)

    def centres(self):
        return MC_MIN * np.exp(self.log_step * np.arange(self.n_mc))

    def cell_of(self, mc):
        return np.clip(np.floor(np.log(np.asarray(mc) / MC_MIN) / self.log_step + 0.5), 0,
                       self.n_mc - 1).astype(np.int64)

    def cell_bounds(self, m):
        lo = MC_MIN * math.exp(self.log_step * (m - 0.5))
        hi = MC_MIN * math.exp(self.log_step * (m + 0.5))
        return max(lo, MC_MIN), min(hi, MC_MAX)

    def fine(self, m, per_cell=8):
        """per_cell fine chirp masses log-spaced inside cell m (cell-centred)."""
        lo, hi = self.cell_bounds(m)
        q = (np.arange(per_cell) + 0.5) / per_cell
        return lo * (hi / lo) ** q

    def fine_of_regions(self, cells, per_cell=8):
        """Fine chirp masses [..., per_cell] of an array of cells."""
        cells = np.asarray(cells)
        out = np.stack([self.fine(int(m), per_cell) for m in cells.ravel()]) if cells.size else \
            np.zeros((0, per_cell))
        return out.reshape(cells.shape + (per_cell,))


def region_of(layout, grid, mc, f):
    """(cell, sub-band) of injections (Mc, f at t0)."""
    b = np.clip(np.floor(np.asarray(f) - layout.band_lo), 0, layout.n_sub - 1).astype(np.int64)
    f0 = layout.band_lo + b + 0.5
    mc_star = np.asarray(mc) * (np.asarray(f) / f0) ** (8.0 / 5.0)
    return grid.cell_of(mc_star), b


def templates(layout, mcs, subs):
    """Template arrays (mc, f0, f_lo, df, K, f_max) of chirp masses mcs in sub-bands subs."""
    mcs = np.asarray(mcs, np.float64).ravel()
    b = np.asarray(subs, np.float64).ravel()
    n = len(mcs)
    return (mcs, layout.band_lo + b + 0.5, layout.band_lo + b, np.full(n, 1.0 / layout.t_coh),
            np.full(n, layout.K, np.int32), np.full(n, layout.band_hi))


def workload(layout, strain, mcs, subs, name="proposal"):
    """One draw's segments x the given templates (template-major full product)."""
    mc, f0, f_lo, df, K, fmax = templates(layout, mcs, subs)
    off = np.arange(layout.n_seg, dtype=np.int64) * layout.L
    return Workload(name=name, strain=np.asarray(strain), seg_offset=off,
                    seg_len=np.full(layout.n_seg, layout.L, np.int64),
                    seg_fs=np.full(layout.n_seg, layout.fs),
                    seg_t=np.arange(layout.n_seg, dtype=np.float64) * layout.t_coh,
                    mc=mc, f0=f0, f_lo=f_lo, df=df, n_bins=K, f_max=fmax, tol=1e-6)


def draw_numpy(layout, grid, region, seed, snr=20.0):
    """One draw: N(0,1) noise over the layout plus, when region = (m, b) is given,
    a 0PN chirp placed in that region (f uniform in the sub-band, Mc* log-uniform in
    the cell, phi0 uniform) scaled to optimal SNR snr.  Draw order: noise, then f,
    the cell position, phi0.  Returns (strain float64, (Mc, f, phi0, amplitude))."""
    rng = np.random.default_rng(seed)
    x = rng.standard_normal(layout.samples)
    if region is None:
        return x, None
    m, b = region
    f = layout.band_lo + b + rng.uniform()
    lo, hi = grid.cell_bounds(int(m))
    mc_star = lo * (hi / lo) ** rng.uniform()
    mc = mc_star * ((layout.band_lo + b + 0.5) / f) ** (8.0 / 5.0)
    phi0 = rng.uniform(0.0, 2.0 * math.pi)
    t = np.arange(layout.samples) / layout.fs
    h = injection(t, f, mc, 1.0, phi0=phi0, f_stop=0.45 * layout.fs)
    amp = snr / math.sqrt(float(np.sum(h * h)))
    return x + amp * h, (mc, f, phi0, amp)


# ----------------------------------------------------------- device draws --

def draw_injections(gen, layout, grid, regions, snr_lo=4.0, snr_hi=20.0):
    """Injection parameters placed in the given (cell, sub-band) regions, drawn on
    gen's device: f uniform in the sub-band, Mc* log-uniform in the cell,
    Mc = Mc* (f0_b / f)^{8/5}, phi0 uniform, SNR uniform in [snr_lo, snr_hi]."""
    import torch
    dev = gen.device
    m, b = (np.asarray(a) for a in regions)
    D = len(m)
    u = torch.rand(D, 4, generator=gen, device=dev, dtype=torch.float64)
    bt = torch.as_tensor(b, device=dev, dtype=torch.float64)
    f = layout.band_lo + bt + u[:, 0]
    bounds = np.array([grid.cell_bounds(int(mm)) for mm in m]).reshape(D, 2)
    lo = torch.as_tensor(bounds[:, 0], device=dev)
    hi = torch.as_tensor(bounds[:, 1], device=dev)
    mc_star = lo * (hi / lo) ** u[:, 1]
    mc = mc_star * ((layout.band_lo + bt + 0.5) / f) ** (8.0 / 5.0)
    phi0 = 2.0 * math.pi * u[:, 2]
    snr = snr_lo + (snr_hi - snr_lo) * u[:, 3]
    return mc, f, phi0, snr


def chirp_waveform(layout, t, mc, f, phi0):
    """Unit-amplitude real 0PN chirps cos(Phi) [D][N] at times t [N] (device, float64):
    Phi of Eq. (phi) relative to t0 plus phi0, zero past coalescence or above 0.45 fs.
    beta of Eq. (beta) per draw comes from the numpy definition in synth."""
    import torch
    b = torch.as_tensor(chirp_beta(mc.cpu().numpy(), f.cpu().numpy()), device=t.device)[:, None]
    y = (8.0 / 3.0) * b * t[None, :]
    ok = y < 1.0
    u = torch.clamp(1.0 - y, min=1e-300)
    ph = (6.0 * math.pi / 5.0) * (f[:, None] / b) * (-torch.expm1(0.625 * torch.log(u))) + phi0[:, None]
    ok &= f[:, None] * u ** (-0.375) <= 0.45 * layout.fs
    return torch.where(ok, torch.cos(ph), torch.zeros_like(ph))


def make_strain(gen, layout, D, inj=None, dtype=None):
    """D draws of N(0,1) noise [D][samples] on gen's device, plus the injections
    (Mc, f, phi0, snr) scaled to their optimal SNR (white noise: rho^2 = sum h^2)."""
    import torch
    dtype = dtype or torch.float32
    dev = gen.device
    x = torch.randn(D, layout.samples, generator=gen, device=dev, dtype=dtype)
    if inj is not None:
        mc, f, phi0, snr = inj
        t = torch.arange(layout.samples, device=dev, dtype=torch.float64) / layout.fs
        for i0 in range(0, D, 64):
            i1 = min(D, i0 + 64)
            h = chirp_waveform(layout, t, mc[i0:i1], f[i0:i1], phi0[i0:i1])
            e = torch.sqrt(torch.clamp((h * h).sum(dim=1), min=1e-300))
            x[i0:i1] += (h * (snr[i0:i1] / e)[:, None]).to(dtype)
    return x
