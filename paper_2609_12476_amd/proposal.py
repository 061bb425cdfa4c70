"""Learned proposal: rank coarse (chirp-mass cell, sub-band) regions for
refinement on a finer chirp-mass grid.

Pipeline (every numeric step runs in the gfx950 library; torch provides
device buffers, the random draws of the synthetic inputs and the top-k
selection bookkeeping):

  coarse grid   n_mc chirp masses log-spaced over [5e-4, 1e-1] Msun x 20 one-hertz
                sub-bands (f0 at the centre), 120 segments of 30 s at 256 Hz;
                semicoherent_sum gives S[template][bin] and N_used.
  features      nr_mlp_region_features: 8 neighbouring chirp masses x 8 bins
                around the template's loudest bin, z = (S/(L sigma^2) - N)/sqrt(N).
  network       64-256-256-1 (nr_mlp_*), trained with BCE + Adam on
                injections the pipeline generates, against noise-only draws.
  refinement    the top-k regions' fine templates (8 per coarse cell,
                log-spaced inside the cell) are searched; the exhaustive fine
                grid is the fallback and the reference it is scored against.

Region and label convention: a region is (coarse cell m, sub-band b); an
injection (Mc, f) belongs to the region whose cell contains
Mc* = Mc (f / f0_b)^{8/5}, f0_b the centre of the sub-band holding f, since
beta(f0_b, Mc*) = beta(f, Mc) (Eq. (beta)): the template with that beta at
f0_b resamples the chirp exactly.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

from . import nufft_resample as nr
from .mlp import Mlp, nr_mlp_region_features

MC_MIN, MC_MAX = 5e-4, 1e-1
BAND_LO, N_SUB = 40.0, 20
FS, T_COH, N_SEG = 256.0, 30.0, 120
L_SEG = int(FS * T_COH)
WORKSPACE = 96 << 30     # device workspace cap of the proposal plans (many draws at once)
T_SUN = 1.3271244e20 / 299792458.0 ** 3


def beta_of(mc, f0):
    return (96.0 / 5.0) * math.pi ** (8.0 / 3.0) * (T_SUN * mc) ** (5.0 / 3.0) * f0 ** (8.0 / 3.0)


@dataclass
class Grid:
    """Coarse chirp-mass grid: n_mc cell centres log-spaced over the range; cell m spans
    [edge_m, edge_{m+1}) with edges half a log step from the centres (clipped to the range)."""
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


def region_of(grid, mc, f):
    """(cell, sub-band) of an injection (Mc, f at t0)."""
    b = np.clip(np.floor(np.asarray(f) - BAND_LO), 0, N_SUB - 1).astype(np.int64)
    f0 = BAND_LO + b + 0.5
    mc_star = np.asarray(mc) * (np.asarray(f) / f0) ** (8.0 / 5.0)
    return grid.cell_of(mc_star), b


# ----------------------------------------------------------------------------
# Synthetic draws on the GPU (inputs, not part of the resampling arithmetic)
# ----------------------------------------------------------------------------

def chirp_waveform(t, mc, f, phi0, dtype):
    """Unit-amplitude 0PN chirp cos(Phi) per draw: Phi of Eq. (phi) relative to t0,
    zero past coalescence or above 0.45 fs.  t [N] (s), mc/f/phi0 [D] tensors."""
    import torch
    b = beta_of_t(mc, f)[:, None]
    y = (8.0 / 3.0) * b * t[None, :]
    ok = y < 1.0
    u = torch.clamp(1.0 - y, min=1e-300)
    ph = (6.0 * math.pi / 5.0) * (f[:, None] / b) * (-torch.expm1(0.625 * torch.log(u))) + phi0[:, None]
    fr = f[:, None] * u ** (-0.375)
    ok &= fr <= 0.45 * FS
    return torch.where(ok, torch.cos(ph), torch.zeros_like(ph)).to(dtype)


def beta_of_t(mc, f0):
    return (96.0 / 5.0) * math.pi ** (8.0 / 3.0) * (T_SUN * mc) ** (5.0 / 3.0) * f0 ** (8.0 / 3.0)


def draw_injections(gen, regions, grid, snr_lo=4.0, snr_hi=20.0):
    """Injection parameters placed in the given (cell, sub-band) regions: f uniform in the
    sub-band, Mc* log-uniform in the cell, Mc = Mc* (f0_b/f)^{8/5}, phi0 uniform, SNR uniform."""
    import torch
    dev = gen.device
    m, b = regions
    D = len(m)
    u = torch.rand(D, 4, generator=gen, device=dev, dtype=torch.float64)
    f = BAND_LO + torch.as_tensor(b, device=dev, dtype=torch.float64) + u[:, 0]
    lo = torch.as_tensor([grid.cell_bounds(int(mm))[0] for mm in m], device=dev, dtype=torch.float64)
    hi = torch.as_tensor([grid.cell_bounds(int(mm))[1] for mm in m], device=dev, dtype=torch.float64)
    mc_star = lo * (hi / lo) ** u[:, 1]
    f0 = BAND_LO + torch.as_tensor(b, device=dev, dtype=torch.float64) + 0.5
    mc = mc_star * (f0 / f) ** (8.0 / 5.0)
    phi0 = 2.0 * math.pi * u[:, 2]
    snr = snr_lo + (snr_hi - snr_lo) * u[:, 3]
    return mc, f, phi0, snr


def make_strain(gen, D, inj=None, dtype=None):
    """D draws of 1 h N(0,1) noise [D][N_SEG*L_SEG], plus the injections (Mc, f, phi0, snr)
    scaled to their optimal SNR (white noise: rho^2 = sum h^2)."""
    import torch
    dtype = dtype or torch.float32
    dev = gen.device
    N = N_SEG * L_SEG
    x = torch.randn(D, N, generator=gen, device=dev, dtype=dtype)
    if inj is not None:
        mc, f, phi0, snr = inj
        t = torch.arange(N, device=dev, dtype=torch.float64) / FS
        for i0 in range(0, D, 64):
            i1 = min(D, i0 + 64)
            h = chirp_waveform(t, mc[i0:i1], f[i0:i1], phi0[i0:i1], torch.float64)
            e = torch.sqrt(torch.clamp((h * h).sum(dim=1), min=1e-300))
            x[i0:i1] += (h * (snr[i0:i1] / e)[:, None]).to(dtype)
    return x


# ----------------------------------------------------------------------------
# Plans
# ----------------------------------------------------------------------------

def _segments(D):
    off = (np.arange(D)[:, None] * (N_SEG * L_SEG) + np.arange(N_SEG)[None, :] * L_SEG).ravel()
    t = np.tile(np.arange(N_SEG) * T_COH, D)
    return nr.make_segments(off, np.full(D * N_SEG, L_SEG), np.full(D * N_SEG, FS), t)


def _templates(mcs, subbands):
    mcs = np.asarray(mcs, np.float64)
    b = np.asarray(subbands, np.float64)
    n = len(mcs)
    return nr.make_templates(mcs, BAND_LO + b + 0.5, BAND_LO + b, np.full(n, 1.0 / T_COH),
                             np.full(n, 30, np.int32), np.full(n, BAND_LO + N_SUB))


class WindowPlan:
    """D draw slots; slot d searches the 8-cell chirp-mass window around its region
    (cells clamp(m-3..m+4) of sub-band b) over its own 120 segments.  Template (i, d)
    is window position i of slot d, stored at i * D + d so the feature builder sees an
    8 x D grid whose row 3 is each slot's own cell."""

    def __init__(self, grid, regions, tol=1e-6, **kw):
        m, b = (np.asarray(a) for a in regions)
        D = len(m)
        centres = grid.centres()
        win = np.clip(m[None, :] + np.arange(-3, 5)[:, None], 0, grid.n_mc - 1)  # [8][D]
        mcs = centres[win].ravel()
        subs = np.broadcast_to(b[None, :], (8, D)).ravel()
        seg = (np.arange(D)[None, :, None] * N_SEG + np.arange(N_SEG)[None, None, :])
        seg = np.broadcast_to(seg, (8, D, N_SEG)).ravel()
        tm = np.broadcast_to((np.arange(8)[:, None] * D + np.arange(D)[None, :])[:, :, None],
                             (8, D, N_SEG)).ravel()
        inst = nr.make_instances(seg, tm)
        self.D = D
        kw.setdefault("max_workspace_bytes", WORKSPACE)
        self.plan = nr.Plan(_segments(D), _templates(mcs, subs), inst, tol=tol, precision="fp32",
                            strain_length=D * N_SEG * L_SEG, **kw)

    def features(self, strain):
        import torch
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        f = nr_mlp_region_features(stat, used, 8, self.D, 30, 1.0 / L_SEG)
        return f.view(8, self.D, 64)[3].contiguous(), stat, used


class CoarsePlan:
    """D draws x the whole coarse grid (n_mc cells x 20 sub-bands, template (m, b) of draw
    d at (m * 20 + b) * D + d... laid out draw-minor so the feature builder runs per draw)."""

    def __init__(self, grid, D, tol=1e-6, **kw):
        centres = grid.centres()
        n_t = grid.n_mc * N_SUB
        mcs = np.repeat(centres, N_SUB)
        subs = np.tile(np.arange(N_SUB), grid.n_mc)
        # templates ordered draw-major: draw d owns templates [d * n_t, (d + 1) * n_t)
        self.D, self.n_t, self.grid = D, n_t, grid
        segs = _segments(D)
        tmpls = _templates(np.tile(mcs, D), np.tile(subs, D))
        seg = np.broadcast_to((np.arange(D)[:, None, None] * N_SEG + np.arange(N_SEG)[None, None, :]),
                              (D, n_t, N_SEG)).ravel()
        tm = np.broadcast_to((np.arange(D)[:, None] * n_t + np.arange(n_t)[None, :])[:, :, None],
                             (D, n_t, N_SEG)).ravel()
        kw.setdefault("max_workspace_bytes", WORKSPACE)
        self.plan = nr.Plan(segs, tmpls, nr.make_instances(seg, tm), tol=tol, precision="fp32",
                            strain_length=D * N_SEG * L_SEG, **kw)

    def run(self, strain):
        """(features [D][n_t][64], stat [D][n_t][30], n_used [D][n_t])."""
        import torch
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        feats = torch.empty(self.D, self.n_t, 64, dtype=torch.float32, device=strain.device)
        for d in range(self.D):
            nr_mlp_region_features(stat[d * self.n_t * 30:(d + 1) * self.n_t * 30],
                                   used[d * self.n_t:(d + 1) * self.n_t], self.grid.n_mc, N_SUB, 30,
                                   1.0 / L_SEG, feats[d])
        return feats, stat.view(self.D, self.n_t, 30), used.view(self.D, self.n_t)


def zstat(stat, used):
    """Standardised summed power (S/(L sigma^2) - N)/sqrt(N) (0 where N = 0)."""
    import torch
    N = used.to(torch.float64)[..., None]
    z = (stat.to(torch.float64) / L_SEG - N) / torch.sqrt(torch.clamp(N, min=1.0))
    return torch.where(N > 0, z, torch.zeros_like(z))


class FinePlan:
    """D draws x an explicit list of fine templates per draw (same count F per draw)."""

    def __init__(self, mcs, subs, D, tol=1e-6, **kw):
        mcs = np.asarray(mcs).reshape(D, -1)
        subs = np.asarray(subs).reshape(D, -1)
        F = mcs.shape[1]
        self.D, self.F = D, F
        seg = np.broadcast_to((np.arange(D)[:, None, None] * N_SEG + np.arange(N_SEG)[None, None, :]),
                              (D, F, N_SEG)).ravel()
        tm = np.broadcast_to((np.arange(D * F)).reshape(D, F)[:, :, None], (D, F, N_SEG)).ravel()
        kw.setdefault("max_workspace_bytes", WORKSPACE)
        self.plan = nr.Plan(_segments(D), _templates(mcs.ravel(), subs.ravel()),
                            nr.make_instances(seg, tm), tol=tol, precision="fp32",
                            strain_length=D * N_SEG * L_SEG, **kw)

    def max_z(self, strain):
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        z = zstat(stat.view(self.D, self.F, 30), used.view(self.D, self.F))
        return z.amax(dim=2)   # [D][F]


def train(net, x, y, epochs=20, batch=1024, lr=1e-3, seed=0, log=None):
    """Minibatch Adam on (x [N][64], y [N]) device tensors; returns the per-epoch mean loss."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = x.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    hist = []
    for ep in range(epochs):
        perm = torch.randperm(N, generator=g).to(x.device)
        tot = torch.zeros((), dtype=torch.float64, device=x.device)
        nb = 0
        for i0 in range(0, N - batch + 1, batch):
            idx = perm[i0:i0 + batch]
            net.train_step(x[idx].contiguous(), y[idx].contiguous(), lr, loss)
            tot += loss.double()[0]
            nb += 1
        hist.append(float(tot) / max(nb, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f}")
    return hist
