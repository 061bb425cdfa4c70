"""Learned proposal: rank coarse (chirp-mass cell, sub-band) regions and
refine the best ones on a finer chirp-mass grid.

ctypes binding of include/nr_proposal.h (``nr_prop_max_z``, ``nr_prop_topk``)
plus the host orchestration of the pipeline.  Every numeric step runs in the
gfx950 library; the host builds plans, moves the k selected region indices
to the host to plan their refinement, and keeps torch buffers:

  coarse        semicoherent_sum over n_mc chirp masses x n_sub sub-bands
                (Sec. III.C) gives S[template][bin] and N_used;
  features      nr_mlp_region_features: z of the 8 neighbouring chirp masses
                x 8 bins around each template's loudest bin;
  network       nr_mlp_forward (64-256-256-1, trained with nr_mlp_train_step
                on injections the method generates);
  top-k         nr_prop_topk on the logits (ties to the lower region);
  refine        semicoherent_sum over the selected regions' fine chirp masses
                (per_cell per coarse cell), then nr_prop_max_z per region.
The non-learned ranking takes nr_prop_max_z of each coarse template instead
of the logits; the exhaustive fine grid (every region refined) is the
fallback and the reference the ranking is judged against.
"""
from __future__ import annotations

import ctypes
from ctypes import c_char_p, c_double, c_int32, c_int64, c_void_p

import numpy as np

from synth.proposal import Grid, Layout, templates

from . import nufft_resample as nr
from .mlp import nr_mlp_region_features

WORKSPACE = 96 << 30     # device workspace cap of the proposal plans (many draws at once)

SIGNATURES = {
    "nr_prop_max_z": (c_int32, [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_double, c_void_p,
                                c_void_p, c_void_p]),
    "nr_prop_topk": (c_int32, [c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p]),
    "nr_prop_last_error": (c_char_p, []),
}
_bound = False


def lib():
    global _bound
    L = nr.load()
    if not _bound:
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _bound = True
    return L


def _check(code):
    if code != 0:
        msg = lib().nr_prop_last_error()
        raise nr.NrError(code, msg.decode() if msg else "")


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def _stream(stream):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return c_void_p(s.cuda_stream)


def _need(t, dtype, n, what):
    import torch
    if not (isinstance(t, torch.Tensor) and t.is_cuda and t.dtype == dtype and t.is_contiguous()):
        raise ValueError(f"{what} must be a contiguous {dtype} CUDA tensor")
    if t.numel() < n:
        raise ValueError(f"{what} needs {n} values, has {t.numel()}")


def nr_prop_max_z(stat, n_used, n_groups, group, K, norm, zmax=None, arg=None, stream=None):
    """(zmax [n_groups] float32, arg [n_groups] int32 or None): the largest z of each
    run of `group` templates (device tensors)."""
    import torch
    _need(stat, torch.float32, n_groups * group * K, "stat")
    _need(n_used, torch.int32, n_groups * group, "n_used")
    if zmax is None:
        zmax = torch.empty(n_groups, dtype=torch.float32, device=stat.device)
    _need(zmax, torch.float32, n_groups, "zmax")
    if arg is not None:
        _need(arg, torch.int32, n_groups, "arg")
    _check(lib().nr_prop_max_z(_ptr(stat), _ptr(n_used), int(n_groups), int(group), int(K), float(norm),
                               _ptr(zmax), _ptr(arg), _stream(stream)))
    return zmax, arg


def nr_prop_topk(scores, rows, n, k, idx=None, stream=None):
    """idx [rows][k] int32: the k best items of each row of scores [rows][n] (device)."""
    import torch
    _need(scores, torch.float32, rows * n, "scores")
    if idx is None:
        idx = torch.empty(rows, k, dtype=torch.int32, device=scores.device)
    _need(idx, torch.int32, rows * k, "idx")
    _check(lib().nr_prop_topk(_ptr(scores), int(rows), int(n), int(k), _ptr(idx), _stream(stream)))
    return idx


# ----------------------------------------------------------------------------
# Plans over D draws of a layout (draw d owns strain [d * samples, (d + 1) * samples))
# ----------------------------------------------------------------------------

def _segments(layout, D):
    off = (np.arange(D)[:, None] * layout.samples + np.arange(layout.n_seg)[None, :] * layout.L).ravel()
    t = np.tile(np.arange(layout.n_seg) * layout.t_coh, D)
    return nr.make_segments(off, np.full(D * layout.n_seg, layout.L), np.full(D * layout.n_seg, layout.fs), t)


def _draw_plan(layout, mcs, subs, D, tol, kw):
    """Plan of D draws x F templates per draw (mcs, subs [D][F]); template (d, f) at
    d * F + f, instances of one template consecutive over its draw's segments."""
    mcs = np.asarray(mcs, np.float64).reshape(D, -1)
    subs = np.asarray(subs).reshape(D, -1)
    F = mcs.shape[1]
    S = layout.n_seg
    seg = np.broadcast_to(np.arange(D)[:, None, None] * S + np.arange(S)[None, None, :], (D, F, S)).ravel()
    tm = np.broadcast_to(np.arange(D * F).reshape(D, F)[:, :, None], (D, F, S)).ravel()
    kw = dict(kw)
    kw.setdefault("max_workspace_bytes", WORKSPACE)
    return nr.Plan(_segments(layout, D), nr.make_templates(*templates(layout, mcs.ravel(), subs.ravel())),
                   nr.make_instances(seg, tm), tol=tol, precision="fp32",
                   strain_length=D * layout.samples, **kw), F


class WindowPlan:
    """One slot per given region (m, b); slot d searches the 8-cell chirp-mass window
    clamp(m-3..m+4) of sub-band b over its own draw.  Template (i, d) is window row i
    of slot d, stored at i * D + d, so the feature builder sees an 8 x D grid whose
    row 3 is each slot's own cell: the training features of the regions."""

    def __init__(self, layout, grid, regions, tol=1e-6, **kw):
        m, b = (np.asarray(a) for a in regions)
        D = len(m)
        win = np.clip(m[None, :] + np.arange(-3, 5)[:, None], 0, grid.n_mc - 1)  # [8][D]
        mcs = grid.centres()[win].ravel()
        subs = np.broadcast_to(b[None, :], (8, D)).ravel()
        S = layout.n_seg
        seg = np.broadcast_to(np.arange(D)[None, :, None] * S + np.arange(S)[None, None, :], (8, D, S)).ravel()
        tm = np.broadcast_to((np.arange(8)[:, None] * D + np.arange(D)[None, :])[:, :, None], (8, D, S)).ravel()
        kw.setdefault("max_workspace_bytes", WORKSPACE)
        self.layout, self.D = layout, D
        self.plan = nr.Plan(_segments(layout, D), nr.make_templates(*templates(layout, mcs, subs)),
                            nr.make_instances(seg, tm), tol=tol, precision="fp32",
                            strain_length=D * layout.samples, **kw)

    def features(self, strain):
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        f = nr_mlp_region_features(stat, used, 8, self.D, self.layout.K, self.layout.norm)
        return f.view(8, self.D, 64)[3].contiguous(), stat, used

    def close(self):
        self.plan.close()


class CoarsePlan:
    """D draws x the whole coarse grid: template (m, b) of draw d at
    d * R + m * n_sub + b, R = n_mc * n_sub regions per draw."""

    def __init__(self, layout, grid, D, tol=1e-6, **kw):
        R = grid.n_mc * layout.n_sub
        mcs = np.tile(np.repeat(grid.centres(), layout.n_sub), D)
        subs = np.tile(np.tile(np.arange(layout.n_sub), grid.n_mc), D)
        self.layout, self.grid, self.D, self.R = layout, grid, D, R
        self.plan, _ = _draw_plan(layout, mcs, subs, D, tol, kw)

    def run(self, strain):
        """(features [D][R][64], stat [D * R * K], n_used [D * R])."""
        import torch
        lay = self.layout
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        feats = torch.empty(self.D, self.R, 64, dtype=torch.float32, device=strain.device)
        step = self.R * lay.K
        for d in range(self.D):
            nr_mlp_region_features(stat[d * step:(d + 1) * step], used[d * self.R:(d + 1) * self.R],
                                   self.grid.n_mc, lay.n_sub, lay.K, lay.norm, feats[d])
        return feats, stat, used

    def max_z(self, stat, used):
        """Largest z of each coarse template, [D][R] (the non-learned score)."""
        z, _ = nr_prop_max_z(stat, used, self.D * self.R, 1, self.layout.K, self.layout.norm)
        return z.view(self.D, self.R)

    def close(self):
        self.plan.close()


class FinePlan:
    """D draws x F fine templates per draw (mcs, subs [D][F]); max_z gives the largest
    z of every group of `group` consecutive fine templates."""

    def __init__(self, layout, mcs, subs, D, tol=1e-6, **kw):
        self.layout, self.D = layout, D
        self.plan, self.F = _draw_plan(layout, mcs, subs, D, tol, kw)

    def max_z(self, strain, group=1):
        stat, used = self.plan.semicoherent_sum(strain.view(-1))
        z, _ = nr_prop_max_z(stat, used, self.D * self.F // group, group, self.layout.K, self.layout.norm)
        return z.view(self.D, self.F // group)

    def close(self):
        self.plan.close()


def rank(net, feats, k):
    """Top-k regions [D][k] (int32, device) of each draw by the network's logits."""
    D, R = feats.shape[0], feats.shape[1]
    logits = net.forward(feats.reshape(D * R, 64))
    return nr_prop_topk(logits, D, R, k), logits.view(D, R)


def rank_max_z(zc, k):
    """Top-k regions [D][k] of each draw by the largest coarse z (the non-learned ranking)."""
    D, R = zc.shape
    return nr_prop_topk(zc.contiguous(), D, R, k)


def refine(layout, grid, strain, top, per_cell=8, **kw):
    """Best fine z [D][k] of each selected region: top [D][k] region indices
    m * n_sub + b (device or host); strain [D][samples] (device)."""
    import torch
    sel = top.cpu().numpy() if isinstance(top, torch.Tensor) else np.asarray(top)
    D, k = sel.shape
    m, b = sel // layout.n_sub, sel % layout.n_sub
    mcs = grid.fine_of_regions(m, per_cell).reshape(D, k * per_cell)
    subs = np.repeat(b, per_cell, axis=1)
    fp = FinePlan(layout, mcs, subs, D, **kw)
    try:
        return fp.max_z(strain, group=per_cell)
    finally:
        fp.close()


def train(net, x, y, epochs=20, batch=1024, lr=1e-3, seed=0, log=None, val=None):
    """Minibatch Adam on (x [N][64], y [N]) device tensors; returns the per-epoch mean
    training loss.  val = (xv, yv): after every epoch the validation loss is taken
    and the parameters of the epoch with the lowest one are kept (early stopping;
    the network then holds them with fresh Adam moments); the per-epoch validation
    losses are appended to the returned history as {"val": [...], "best_epoch": e}."""
    import torch
    g = torch.Generator(device="cpu").manual_seed(seed)
    N = x.shape[0]
    loss = torch.empty(1, dtype=torch.float32, device=x.device)
    hist, vhist, best = [], [], (float("inf"), -1, None)
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
        msg = f"epoch {ep}: loss {hist[-1]:.4f}"
        if val is not None:
            vl = float(net.loss(*val))
            vhist.append(vl)
            msg += f", validation {vl:.4f}"
            if vl < best[0]:
                best = (vl, ep, net.get_params())
        if log:
            log(msg)
    if val is not None and best[2] is not None:
        net.set_params(best[2])
        return {"train": hist, "val": vhist, "best_epoch": best[1]}
    return hist


__all__ = ["Grid", "Layout", "WindowPlan", "CoarsePlan", "FinePlan", "nr_prop_max_z", "nr_prop_topk", "rank",
           "rank_max_z", "refine", "train"]
