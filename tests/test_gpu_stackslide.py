"""Parity of the stack-slide kernels (through the C ABI) with the oracle.

Track tables (end of track, beta template and bin of every lag) bit-exact;
weights' running sums to 1e-12 relative; n_sigma to 2e-6 absolute (float32
output; the kernel accumulates in FP64) on the same power array, in both
power layouts; the transpose bit-exact.  End to end: the spectra of an
injected chirp computed by the NUFFT path put the largest statistic on the
injection's own track.
"""
import math
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import stackslide as oss

pytestmark = pytest.mark.gpu

BETAS, _ = synth.beta_bank(69)
NS_TOL = 2e-6


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _plan(n_seg, n_bins, mcs, S, L, layout=0, t_coh=30.0):
    from paper_2609_12476_amd import stackslide as ss
    g = ss.geometry(n_seg=n_seg, n_beta=len(BETAS), n_bins=n_bins, t_coh=t_coh, f_lo=40.0, df=1.0 / t_coh,
                    f_start=40.0, f_max=60.0, norm=2.0 / L, layout=layout)
    return ss.StackSlide(g, BETAS, mcs, S)


def test_tables_match_oracle(gpu):
    say("stack-slide tables")
    mcs = np.array([1e-4, 3e-3, 2e-2, 6e-2, 1e-1, 3e-1])
    n_seg, S = 40, 3
    with _plan(n_seg, 600, mcs, S, 15360) as p:
        k, j, w2, ln = p.tables()
    for c, mc in enumerate(mcs):
        for s in range(S):
            segs = oss.track_grid(mc, 0, s, S, n_seg, 30.0, BETAS, 40.0, 1.0 / 30.0, 600, 40.0, 60.0)
            assert ln[c, s] == len(segs), (mc, s)
            ks = np.array([q[1] for q in segs], np.int32)
            js = np.array([q[2] for q in segs], np.int32)
            assert np.array_equal(k[c, s, :len(segs)], ks), (mc, s)
            assert np.array_equal(j[c, s, :len(segs)], js), (mc, s)
            f = np.array([q[3] for q in segs])
            cum = np.cumsum(f ** (8.0 / 3.0))
            assert np.allclose(w2[c, s, :len(segs)], cum, rtol=1e-12, atol=0)
    assert ln[0].min() == n_seg and ln[-1].max() < n_seg          # tiny Mc never ends, heavy ones do


# S: start offsets per segment (track families per chirp mass)
@pytest.mark.parametrize("layout,S", [(0, 2), (1, 2), (1, 20)])
def test_n_sigma_matches_oracle(gpu, layout, S):
    import torch
    from paper_2609_12476_amd import stackslide as ss
    say(f"stack-slide n_sigma layout {layout} S {S}")
    n_seg, n_bins, L = 24, 600, 15360
    mcs = np.array([5e-4, 1e-2, 4e-2, 9e-2])
    P = synth.noise_power(len(BETAS), n_seg, n_bins, L, seed=3)
    Pd = torch.from_numpy(P).to(gpu)
    if layout == 1:
        Pd = ss.nr_ss_transpose(Pd, len(BETAS), n_seg, n_bins)
    with _plan(n_seg, n_bins, mcs, S, L, layout=layout) as p:
        ns, used = p.execute(Pd)
        torch.cuda.synchronize()
        ns, used = ns.cpu().numpy(), used.cpu().numpy()
    ref, cnt = oss.n_sigma(P, mcs, S, 30.0, BETAS, 40.0, 1.0 / 30.0, 40.0, 60.0, 2.0 / L)
    assert np.array_equal(used, cnt)
    err = np.abs(ns - ref).max()
    say(f"  max |d n_sigma| = {err:.2e} over {ns.size} tracks (|n_sigma| up to {np.abs(ref).max():.2f})")
    assert err <= NS_TOL * max(1.0, np.abs(ref).max())


@pytest.mark.parametrize("layout,S", [(0, 2), (1, 2), (0, 20)])
def test_segment_range_partial_sums(gpu, layout, S):
    """Sec. VI's partial sums: the statistic accumulated over segment ranges held
    in memory one at a time (ranges of 7, 1, 10 and 6 segments, summed out of
    order) equals the whole-array statistic (float rounding of the partials)
    and the oracle; the segment counts add up exactly."""
    import torch
    from paper_2609_12476_amd import stackslide as ss
    say(f"stack-slide ranges layout {layout} S {S}")
    n_seg, n_bins, L = 24, 600, 15360
    mcs = np.array([5e-4, 1e-2, 4e-2, 9e-2])
    P = synth.noise_power(len(BETAS), n_seg, n_bins, L, seed=5)
    ranges = [(7, 1), (17, 7), (0, 7), (8, 9)]      # (start, count): a partition of [0, 24), out of order
    assert sorted(a for a, _ in ranges) == [0, 7, 8, 17] and sum(c for _, c in ranges) == n_seg
    with _plan(n_seg, n_bins, mcs, S, L, layout=layout) as p:
        full = torch.from_numpy(P).to(gpu)
        if layout == 1:
            full = ss.nr_ss_transpose(full, len(BETAS), n_seg, n_bins)
        ns_full, used_full = p.execute(full)
        ns = torch.zeros_like(ns_full)
        used = torch.zeros_like(used_full)
        for a, c in ranges:
            part = torch.from_numpy(np.ascontiguousarray(P[:, a:a + c, :])).to(gpu)
            if layout == 1:
                part = ss.nr_ss_transpose(part, len(BETAS), c, n_bins)
            p.execute_range(part, a, c, ns, used)
        torch.cuda.synchronize()
        ns, used = ns.cpu().numpy(), used.cpu().numpy()
        ns_full, used_full = ns_full.cpu().numpy(), used_full.cpu().numpy()
    ref, cnt = oss.n_sigma(P, mcs, S, 30.0, BETAS, 40.0, 1.0 / 30.0, 40.0, 60.0, 2.0 / L)
    assert np.array_equal(used, used_full) and np.array_equal(used, cnt)
    scale = max(1.0, np.abs(ref).max())
    assert np.abs(ns - ns_full).max() <= 4 * NS_TOL * scale
    assert np.abs(ns - ref).max() <= 4 * NS_TOL * scale
    from paper_2609_12476_amd import NrError
    with pytest.raises(NrError):
        with _plan(n_seg, n_bins, mcs, S, L, layout=layout) as p:
            p.execute_range(torch.from_numpy(P).to(gpu), 20, 5, torch.zeros(len(mcs), n_seg * S, device=gpu))


def test_transpose_is_exact(gpu):
    import torch
    from paper_2609_12476_amd import stackslide as ss
    P = synth.noise_power(5, 37, 71, 100, seed=4)
    T = ss.nr_ss_transpose(torch.from_numpy(P).to(gpu), 5, 37, 71)
    torch.cuda.synchronize()
    assert np.array_equal(T.cpu().numpy().reshape(5, 71, 37), P.transpose(0, 2, 1))


def test_injection_found_end_to_end(gpu):
    """Spectra of an injected chirp from the NUFFT path, then the stack-slide:
    the injection's (Mc, t0) gives the largest statistic, and sampled tracks
    match the oracle on the same power."""
    import torch
    from paper_2609_12476_amd import Plan
    say("stack-slide end to end")
    mc, t0 = 1e-1, 45.0
    fs, t_coh = 256.0, 30.0
    w = synth.paper_bank(hours=0.3, fs=fs, t_coh=t_coh, inject=(mc, t0, 0.5, 0.3)).as_float32_strain()
    n_seg, K, L = w.n_seg, int(w.n_bins[0]), int(w.seg_len[0])
    with Plan.from_workload(w, precision="fp32", tol=1e-6) as pl:
        x = pl.strain_tensor(w.strain, gpu)
        _, pw, valid = pl.execute(x, want=("power", "valid"))
        assert bool(valid.all())
    S = 4
    mcs = mc * np.array([0.94, 0.97, 1.0, 1.03, 1.06])
    with _plan(n_seg, K, mcs, S, L) as p:
        ns, used = p.execute(pw)
        torch.cuda.synchronize()
        ns = ns.cpu().numpy()
    i0 = int(math.ceil(t0 / t_coh))
    s_true = int(round((i0 * t_coh - t0) / t_coh * S))
    c_best, q_best = np.unravel_index(np.argmax(ns), ns.shape)
    say(f"  best track (c={c_best}, i0={q_best // S}, s={q_best % S}) n_sigma {ns.max():.1f}")
    assert (c_best, q_best) == (2, i0 * S + s_true)
    P = pw.cpu().numpy().astype(np.float64).reshape(len(BETAS), n_seg, K)
    rng = np.random.default_rng(5)
    cand = [(int(c), int(q) // S, int(q) % S) for c, q in
            zip(rng.integers(0, len(mcs), 40), rng.integers(0, n_seg * S, 40))] + [(2, i0, s_true)]
    ref, _ = oss.n_sigma(P, mcs, S, t_coh, BETAS, 40.0, 1.0 / t_coh, 40.0, 60.0, 2.0 / L, tracks=cand)
    for (c, i0_, s) in cand:
        q = i0_ * S + s
        assert abs(ns[c, q] - ref[c, q]) <= NS_TOL * max(1.0, abs(ref[c, q])), (c, i0_, s)


def test_fullsize_paper_1h_sampled(gpu):
    """The benchmark's configuration: the paper's 1 h spectra (120 segments x 69
    beta x 600 bins) from the NUFFT path, 2048 chirp masses x 120 x 8 start
    times in the [beta][bin][segment] layout; sampled tracks against the
    oracle on the same power, and both layouts equal."""
    import torch
    from paper_2609_12476_amd import Plan
    from paper_2609_12476_amd import stackslide as ss
    say("stack-slide full size")
    w = synth.paper_bank(hours=1.0).as_float32_strain()
    n_seg, K, L = w.n_seg, int(w.n_bins[0]), int(w.seg_len[0])
    with Plan.from_workload(w, precision="fp32", tol=1e-6) as pl:
        x = pl.strain_tensor(w.strain, gpu)
        _, pw, _ = pl.execute(x, want=("power",))
    pt = ss.nr_ss_transpose(pw, len(BETAS), n_seg, K)
    mcs = synth.log_spaced_mc(2048)
    S = 8
    res = []
    for layout, P in ((1, pt), (0, pw)):
        with _plan(n_seg, K, mcs, S, L, layout=layout) as p:
            ns, used = p.execute(P)
            torch.cuda.synchronize()
            res.append((ns.cpu().numpy(), used.cpu().numpy()))
    assert np.array_equal(res[0][0], res[1][0]) and np.array_equal(res[0][1], res[1][1])
    ns, used = res[0]
    Ph = pw.cpu().numpy().astype(np.float64).reshape(len(BETAS), n_seg, K)
    rng = np.random.default_rng(13)
    cand = [(int(c), int(q) // S, int(q) % S) for c, q in
            zip(rng.integers(0, len(mcs), 200), rng.integers(0, n_seg * S, 200))]
    ref, cnt = oss.n_sigma(Ph, mcs, S, 30.0, BETAS, 40.0, 1.0 / 30.0, 40.0, 60.0, 2.0 / L, tracks=cand)
    err = 0.0
    for (c, i0, s) in cand:
        q = i0 * S + s
        assert used[c, q] == cnt[c, q], (c, i0, s)
        err = max(err, abs(ns[c, q] - ref[c, q]))
    say(f"  200 sampled tracks: max |d n_sigma| {err:.2e}")
    assert err <= NS_TOL * max(1.0, float(np.abs(ref[~np.isnan(ref)]).max()))
