"""Parity of the gfx950 path (through the C ABI) with the oracle.

Bounds: relative l2 over an instance's bins <= 1e-9 in FP64 and <= 1e-5 in
FP32; segment sums <= 1e-9 (FP64) and <= 1e-4 (FP32) relative l2 per
template; validity flags and segment counts bit-exact.
"""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu

FP32_SPEC = 1e-5
FP32_SUM = 1e-4
FP64_SPEC = 1e-9


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def run_plan(w, dev, **kw):
    import torch
    from paper_2609_12476_amd import Plan, complex_view
    with Plan.from_workload(w, **kw) as p:
        x = p.strain_tensor(w.strain, dev)
        sp, pw, valid = p.execute(x)
        torch.cuda.synchronize()
        X = complex_view(sp).cpu().numpy().astype(np.complex128)
        return X, pw.cpu().numpy().astype(np.float64), valid.cpu().numpy(), p.bin_offsets(), p.classes()


def run_sum(w, dev, seg_weight=None, **kw):
    import torch
    from paper_2609_12476_amd import Plan
    with Plan.from_workload(w, **kw) as p:
        x = p.strain_tensor(w.strain, dev)
        sw = None if seg_weight is None else torch.tensor(seg_weight, dtype=torch.float64, device=dev)
        stat, used = p.semicoherent_sum(x, sw)
        torch.cuda.synchronize()
        return stat.cpu().numpy().astype(np.float64), used.cpu().numpy(), p.stat_offsets()


def rel(a, b):
    nb = np.linalg.norm(b)
    return np.linalg.norm(a - b) / nb if nb > 0 else np.linalg.norm(a)


def per_instance_errors(X, Xr, off, ok):
    errs = []
    for i in range(len(off) - 1):
        a, b = X[off[i]:off[i + 1]], Xr[off[i]:off[i + 1]]
        if ok[i]:
            errs.append(rel(a, b))
        else:
            assert not np.any(a), f"invalid instance {i} not zero"
    return np.array(errs)


# ------------------------------------------------------------ single segment --

@pytest.mark.parametrize("method", ["fused", "staged", "cellrun", "direct"])
def test_single_segment_fp64(gpu, method):
    say(f"single_segment fp64 {method}")
    w = synth.single_segment()
    Xr, off, ok = oracle.spectra(w)
    X, P, valid, off_g, cls = run_plan(w, gpu, precision="fp64", method=method, tol=1e-9)
    assert np.array_equal(off, off_g) and valid[0] == 1
    assert cls[0].n == 1200 and cls[0].fp64 == 1
    e = rel(X, Xr)
    say(f"  rel l2 = {e:.3e} (w={cls[0].w}, degree={cls[0].degree})")
    assert e <= FP64_SPEC
    assert np.allclose(P, np.abs(X) ** 2, rtol=1e-12, atol=0)


@pytest.mark.parametrize("method", ["fused", "staged", "cellrun", "direct"])
def test_single_segment_fp32(gpu, method):
    say(f"single_segment fp32 {method}")
    w = synth.single_segment()
    Xr, off, ok = oracle.spectra(w)
    X, P, valid, _, cls = run_plan(w, gpu, precision="fp32", method=method, tol=1e-6)
    e = rel(X, Xr)
    say(f"  rel l2 = {e:.3e}")
    assert e <= FP32_SPEC
    assert np.allclose(P, np.abs(X) ** 2, rtol=1e-6, atol=1e-6 * np.max(P))


def test_analytic_chirp_collapse_on_gpu(gpu):
    say("analytic chirp collapse")
    L, fs, A = 7680, 256.0, 0.05
    t = np.arange(L) / fs
    w = synth.single_segment()
    w.strain = synth.injection(t, 50.0, 1e-2, A, analytic=True)
    X, P, valid, _, _ = run_plan(w, gpu, precision="fp64", tol=1e-10, strain_complex=True)
    assert np.argmax(P) == 300
    assert abs(P[300] / (L * A / 2) ** 2 - 1.0) < 1e-9


# ------------------------------------------------------------ semicoherent ----

@pytest.mark.parametrize("prec,method", [("fp32", "fused"), ("fp32", "staged"), ("fp32", "cellrun"),
                                         ("fp32", "direct"), ("fp64", "fused"), ("fp64", "staged"),
                                         ("fp64", "cellrun"), ("fp64", "direct")])
def test_semicoherent_small(gpu, prec, method):
    say(f"semicoherent small {prec} {method}")
    w = synth.semicoherent(hours=0.1, n_mc=4, n_sub=3, seed=3, snr=30.0)
    Xr, off, ok = oracle.spectra(w)
    tol = 1e-6 if prec == "fp32" else 1e-10
    X, P, valid, off_g, _ = run_plan(w, gpu, precision=prec, method=method, tol=tol)
    assert np.array_equal(valid, ok) and np.array_equal(off, off_g)
    errs = per_instance_errors(X, Xr, off, ok)
    say(f"  {len(errs)} valid of {w.n_inst}; max rel {errs.max():.3e} median {np.median(errs):.3e}")
    assert errs.max() <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)
    Sr, soff, used_r = oracle.semicoherent(w)
    S, used, soff_g = run_sum(w, gpu, precision=prec, method=method, tol=tol)
    assert np.array_equal(used, used_r) and np.array_equal(soff, soff_g)
    for m in range(w.n_tmpl):
        a, b = S[soff[m]:soff[m + 1]], Sr[soff[m]:soff[m + 1]]
        if used_r[m]:
            assert rel(a, b) <= (FP32_SUM if prec == "fp32" else FP64_SPEC), m
        else:
            assert not np.any(a)


def test_semicoherent_weights_and_accumulation(gpu):
    say("semicoherent weights")
    import torch
    from paper_2609_12476_amd import Plan
    w = synth.semicoherent(hours=0.05, n_mc=3, n_sub=2, seed=8)
    wts = np.linspace(0.25, 2.0, w.n_seg)
    Sr, soff, used_r = oracle.semicoherent(w, seg_weight=wts)
    with Plan.from_workload(w, precision="fp64", tol=1e-10) as p:
        x = p.strain_tensor(w.strain, gpu)
        sw = torch.tensor(wts, dtype=torch.float64, device=gpu)
        stat, used = p.semicoherent_sum(x, sw)
        stat, used = p.semicoherent_sum(x, sw, stat, used)    # accumulates
        torch.cuda.synchronize()
        S = stat.cpu().numpy()
        assert np.array_equal(used.cpu().numpy(), 2 * used_r)
        assert rel(S, 2 * Sr) <= FP64_SPEC


def test_semicoherent_determinism(gpu):
    say("determinism")
    w = synth.semicoherent(hours=0.1, n_mc=4, n_sub=3, seed=5)
    a = run_sum(w, gpu, precision="fp32", tol=1e-6)[0]
    b = run_sum(w, gpu, precision="fp32", tol=1e-6)[0]
    assert np.array_equal(a, b)
    X1 = run_plan(w, gpu, precision="fp32", tol=1e-6)[0]
    X2 = run_plan(w, gpu, precision="fp32", tol=1e-6)[0]
    assert np.array_equal(X1, X2)


# ----------------------------------------------------------------- ragged ----

def test_ragged_batch_auto_precision(gpu):
    say("ragged auto")
    w = synth.ragged_batch(n_inst=30, seed=12)
    Xr, off, ok = oracle.spectra(w)
    X, P, valid, off_g, cls = run_plan(w, gpu, precision="auto")
    assert np.array_equal(off, off_g)
    say(f"  classes: {[(c.fp64, c.w, c.n, c.parts) for c in cls]}")
    for i in range(w.n_inst):
        if not ok[i]:
            continue
        t = w.inst_tol[i]
        bound = max(t, FP32_SPEC) if t >= 1e-6 else max(t, 1e-11)
        e = rel(X[off[i]:off[i + 1]], Xr[off[i]:off[i + 1]])
        assert e <= bound, (i, t, e, w.seg_len[w.inst_seg[i]], w.n_bins[i])


def test_ragged_batch_grouped_launches(gpu):
    """Many kernel classes in one plan run as a few grouped launches; spectra
    and segment sums still match the oracle class by class."""
    import torch
    from paper_2609_12476_amd import Plan, complex_view
    say("ragged grouped launches")
    w = synth.ragged_batch(n_inst=24, seed=21)
    w.inst_tol = np.where(w.inst_tol < 1e-6, 1e-6, w.inst_tol)     # FP32 classes only
    Xr, off, ok = oracle.spectra(w)
    # every template of this batch has one instance: its segment sum is that
    # instance's power
    Sr, soff, used_r = np.abs(Xr) ** 2, off, ok.astype(np.int32)
    with Plan.from_workload(w, precision="fp32") as p:
        cls = p.classes()
        say(f"  {len(cls)} classes, {p.info.n_chunks} spread launches, parts {sorted({c.parts for c in cls})}")
        assert len(cls) > 1 and p.info.n_chunks < len(cls)
        x = p.strain_tensor(w.strain, gpu)
        sp, _, valid = p.execute(x)
        stat, used = p.semicoherent_sum(x)
        torch.cuda.synchronize()
        X = complex_view(sp).cpu().numpy().astype(np.complex128)
        S = stat.cpu().numpy().astype(np.float64)
        used = used.cpu().numpy()
    assert np.array_equal(valid.cpu().numpy(), ok) and np.array_equal(used, used_r)
    # each instance against its own tolerance (FP32 classes: at least 1e-5)
    worst = 0.0
    for i in range(w.n_inst):
        if not ok[i]:
            assert not np.any(X[off[i]:off[i + 1]]), f"invalid instance {i} not zero"
            continue
        t = float(w.inst_tol[i])
        e = rel(X[off[i]:off[i + 1]], Xr[off[i]:off[i + 1]])
        worst = max(worst, e / max(t, FP32_SPEC))
        assert e <= max(t, FP32_SPEC), (i, t, e)
    say(f"  spectra worst error / bound {worst:.3e}")
    # a one-instance template's sum is that instance's power, whose relative
    # error is at most about twice the spectrum's
    for m in range(len(soff) - 1):
        if used_r[m]:
            t = float(w.inst_tol[m])
            e = rel(S[soff[m]:soff[m + 1]], Sr[soff[m]:soff[m + 1]])
            assert e <= (FP32_SUM if t <= 1e-6 else max(FP32_SUM, 3 * t)), (m, t, e)


def test_classes_sharing_templates(gpu):
    """Two FP32 classes (different kernel widths) hold instances of the same
    templates: their segment-sum contributions must all arrive."""
    say("classes sharing templates")
    w = synth.semicoherent(hours=0.1, n_mc=3, n_sub=2, seed=5, snr=25.0)
    w = w.subset(np.arange(w.n_inst))
    w.inst_tol = np.where(np.arange(w.n_inst) % 2 == 0, 1e-6, 1e-5)
    Sr, soff, used_r = oracle.semicoherent(w)
    S, used, _ = run_sum(w, gpu, precision="fp32")
    assert np.array_equal(used, used_r)
    for m in range(len(soff) - 1):
        if used_r[m]:
            assert rel(S[soff[m]:soff[m + 1]], Sr[soff[m]:soff[m + 1]]) <= FP32_SUM


# ------------------------------------------------------------- edge cases ----

@pytest.mark.parametrize("L,K,mc", [(1, 3, 1e-2), (5, 8, 3e-2), (63, 17, 1e-2), (64, 16, 5e-4),
                                    (65, 9, 1e-1), (130, 40, 2e-2), (1000, 1, 1e-2), (257, 101, 0.0)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
@pytest.mark.parametrize("method", ["fused", "cellrun"])
def test_small_and_ragged_sizes(gpu, L, K, mc, prec, method):
    say(f"edge L={L} K={K} mc={mc} {prec} {method}")
    w = synth.random_small(L + K, L, K, mc, f0=50.0, fs=64.0, t_start=3.0)
    Xr, off, ok = oracle.spectra(w)
    X, P, valid, _, _ = run_plan(w, gpu, precision=prec, method=method,
                                 tol=1e-6 if prec == "fp32" else 1e-10)
    assert valid[0] == ok[0] == 1
    assert rel(X, Xr) <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)


@pytest.mark.parametrize("prec,K,n,K_over", [("fp32", 2560, 5120, 2561), ("fp64", 1215, 2430, 1216)])
def test_largest_grid_and_beyond(gpu, prec, K, n, K_over):
    """The largest grid a spreader workgroup's LDS holds (four per-wave grids,
    and in FP64 the 256-entry phase table, in 160 KB: n = 5120 = 2^10 5 in
    FP32, 2430 = 2 3^5 5 in FP64, at sigma 2) matches the oracle; the next
    smooth size is refused with NR_ERR_INVALID_ARG at plan creation."""
    from paper_2609_12476_amd import NrError
    say(f"largest grid {prec}")
    tol = 1e-6 if prec == "fp32" else 1e-10
    w = synth.random_small(77, 6000, K, 2e-2, f0=50.0, fs=256.0)
    Xr, off, ok = oracle.spectra(w)
    X, _, valid, _, cls = run_plan(w, gpu, precision=prec, tol=tol)
    say(f"  grid {cls[0].n}, method {cls[0].method}, error {rel(X, Xr):.2e}")
    assert cls[0].n == n
    assert valid[0] == ok[0] == 1
    assert rel(X, Xr) <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)
    w2 = synth.random_small(78, 6000, K_over, 2e-2, f0=50.0, fs=256.0)
    with pytest.raises(NrError) as e:
        run_plan(w2, gpu, precision=prec, tol=tol)
    assert e.value.code == 1          # NR_ERR_INVALID_ARG


@pytest.mark.parametrize("K", [28, 30, 31, 32, 33, 34, 40, 48, 60, 62, 63, 64, 66, 72])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_cellrun_round_edges(gpu, K, prec):
    """Cell-run instances whose visited cells fall on both sides of one and
    two full rounds of 63 cells (one run per lane but the last), so that a
    round's first run starts where the previous round's last one ended."""
    say(f"cellrun round edges K={K} {prec}")
    w = synth.random_small(100 + K, 2048, K, 3e-2, f0=50.0, fs=64.0, t_start=300.0)
    Xr, off, ok = oracle.spectra(w)
    X, _, valid, _, cls = run_plan(w, gpu, precision=prec, method="cellrun", sigma=2.0,
                                   tol=1e-6 if prec == "fp32" else 1e-10)
    span = oracle.dtau(3e-2, 50.0, 300.0, 64.0, 2048)[-1]
    say(f"  grid {cls[0].n}, about {cls[0].n * span / 32.0 + 1:.1f} cells visited")
    assert valid[0] == ok[0] == 1
    assert rel(X, Xr) <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)


@pytest.mark.parametrize("method", ["fused", "staged", "cellrun"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_complex_strain(gpu, prec, method):
    say(f"complex strain {prec} {method}")
    w = synth.random_small(3, 3000, 64, 2e-2, f0=45.0, fs=128.0, complex_strain=True)
    Xr, off, ok = oracle.spectra(w)
    X, _, _, _, _ = run_plan(w, gpu, precision=prec, method=method,
                             tol=1e-6 if prec == "fp32" else 1e-10)
    assert rel(X, Xr) <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)


def test_identity_map_equals_fft(gpu):
    say("identity = fft")
    L, fs = 512, 128.0
    x = np.random.default_rng(21).standard_normal(L)
    w = synth.pure_tone(L=L, fs=fs, f_lo=0.0, df=fs / L, K=L)
    w.strain = x
    X, _, _, _, _ = run_plan(w, gpu, precision="fp64", tol=1e-11)
    assert rel(X, np.fft.fft(x)) <= FP64_SPEC


@pytest.mark.parametrize("parts", [1, 2, 4, 8, 16])
@pytest.mark.parametrize("sigma", [1.25, 2.0, 3.0])
@pytest.mark.parametrize("method", ["fused", "cellrun"])
def test_parts_and_upsampling(gpu, parts, sigma, method):
    say(f"parts={parts} sigma={sigma} {method}")
    w = synth.single_segment()
    Xr, _, _ = oracle.spectra(w)
    X, _, _, _, cls = run_plan(w, gpu, precision="fp64", tol=1e-9, parts=parts, sigma=sigma, method=method)
    assert cls[0].parts == parts
    assert rel(X, Xr) <= FP64_SPEC


@pytest.mark.parametrize("method", ["fused", "cellrun"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_near_coalescence_uses_tau_kernel(gpu, method, prec):
    """A template so close to coalescence that tau needs the log1p/expm1 form:
    the plan routes it through the tau kernel (staged) and stays exact."""
    import math
    say(f"near coalescence {method} {prec}")
    w = synth.random_small(77, 4096, 64, 1e-1, f0=50.0, fs=64.0, t_start=800.0)
    b = synth.chirp_beta(1e-1, 50.0)
    assert 1 - (8 / 3) * b * (800.0 + 4095 / 64.0) > 0           # still valid at the end
    Xr, off, ok = oracle.spectra(w)
    assert ok[0]
    X, _, valid, _, cls = run_plan(w, gpu, precision=prec, method=method,
                                   tol=1e-6 if prec == "fp32" else 1e-10)
    say(f"  methods {[c.method for c in cls]}, series terms {[c.series_terms for c in cls]}")
    assert valid[0] == 1 and cls[0].method == 1
    assert rel(X, Xr) <= (FP32_SPEC if prec == "fp32" else FP64_SPEC)


def test_invalid_instances_are_zero_and_flagged(gpu):
    say("invalid instances")
    w = synth.semicoherent(hours=0.5, n_mc=3, n_sub=2, seed=9)
    w.mc = np.array([1e-1, 1e-1, 8e-2, 8e-2, 5e-4, 5e-4])    # heavy templates coalesce early
    idx = np.arange(0, w.n_inst, 7)
    sub = w.subset(idx)
    Xr, off, ok = oracle.spectra(sub)
    assert ok.sum() < len(ok) and ok.sum() > 0
    X, P, valid, _, _ = run_plan(sub, gpu, precision="fp32", tol=1e-6)
    assert np.array_equal(valid, ok)
    errs = per_instance_errors(X, Xr, off, ok)
    assert errs.max() <= FP32_SPEC


def test_graph_replay_matches_eager(gpu):
    say("graph replay")
    import torch
    from paper_2609_12476_amd import Plan
    w = synth.semicoherent(hours=0.1, n_mc=4, n_sub=3, seed=13)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pe = Plan.from_workload(w, precision="fp32", tol=1e-6, stream=s)
        pg = Plan.from_workload(w, precision="fp32", tol=1e-6, stream=s, use_graph=True)
        x = pe.strain_tensor(w.strain, gpu)
        sp_e, pw_e, v_e = pe.execute(x)
        st_e, u_e = pe.semicoherent_sum(x)
        s.synchronize()
        sp_g, pw_g, v_g = torch.empty_like(sp_e), torch.empty_like(pw_e), torch.empty_like(v_e)
        st_g, u_g = torch.zeros_like(st_e), torch.zeros_like(u_e)
        for rep in range(4):
            # the program's own eager work between replays
            sp_g.fill_(-1.0)
            pw_g.fill_(-1.0)
            v_g.fill_(7)
            st_g.zero_()
            u_g.zero_()
            pg.execute(x, sp_g, pw_g, v_g)
            pg.semicoherent_sum(x, None, st_g, u_g)
            s.synchronize()
            assert torch.equal(sp_g, sp_e) and torch.equal(pw_g, pw_e) and torch.equal(v_g, v_e), rep
            assert torch.equal(st_g, st_e) and torch.equal(u_g, u_e), rep
        pe.close()
        pg.close()


def test_grouped_graph_replay_matches_eager(gpu):
    """A plan of many classes launched in groups on side streams, captured in a
    graph and replayed: every replay equals the eager launches."""
    say("grouped graph replay")
    import torch
    from paper_2609_12476_amd import Plan
    w = synth.ragged_batch(n_inst=48, seed=23)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        pe = Plan.from_workload(w, precision="auto", stream=s)
        pg = Plan.from_workload(w, precision="auto", stream=s, use_graph=True)
        say(f"  {len(pe.classes())} classes in {pe.info.n_chunks} spread launches")
        assert pe.info.n_chunks < len(pe.classes())
        x = pe.strain_tensor(w.strain, gpu)
        sp_e, pw_e, v_e = pe.execute(x)
        st_e, u_e = pe.semicoherent_sum(x)
        s.synchronize()
        sp_g, pw_g, v_g = torch.empty_like(sp_e), torch.empty_like(pw_e), torch.empty_like(v_e)
        st_g, u_g = torch.zeros_like(st_e), torch.zeros_like(u_e)
        for rep in range(4):
            sp_g.fill_(-1.0)
            pw_g.fill_(-1.0)
            v_g.fill_(7)
            st_g.zero_()
            u_g.zero_()
            pg.execute(x, sp_g, pw_g, v_g)
            pg.semicoherent_sum(x, None, st_g, u_g)
            s.synchronize()
            assert torch.equal(sp_g, sp_e) and torch.equal(pw_g, pw_e) and torch.equal(v_g, v_e), rep
            assert torch.equal(st_g, st_e) and torch.equal(u_g, u_e), rep
        pe.close()
        pg.close()


def test_autotuned_plan_parity_and_cache(gpu, tmp_path):
    say("autotuner")
    w = synth.ragged_batch(n_inst=12, seed=31)
    Xr, off, ok = oracle.spectra(w)
    cache = str(tmp_path / "tune.txt")
    X, _, _, _, cls = run_plan(w, gpu, precision="auto", tune=True, tune_cache=cache)
    lines = open(cache).read().split("\n")
    assert len([l for l in lines if l.strip()]) >= 1
    say(f"  tuned classes: {[(c.fp64, c.w, c.n, c.parts, c.method, c.flush_period) for c in cls]}")
    for i in range(w.n_inst):
        if ok[i]:
            t = w.inst_tol[i]
            bound = max(t, FP32_SPEC) if t >= 1e-6 else max(t, 1e-11)
            assert rel(X[off[i]:off[i + 1]], Xr[off[i]:off[i + 1]]) <= bound
    # a second plan reads the cache and picks the same configurations and FFT plans
    _, _, _, _, cls2 = run_plan(w, gpu, precision="auto", tune=True, tune_cache=cache)
    key = lambda c: (c.parts, c.method, c.flush_period, tuple(c.radix[:c.n_radix]))
    assert [key(c) for c in cls] == [key(c) for c in cls2]
    for c in cls:
        assert int(np.prod(c.radix[:c.n_radix])) == c.n


@pytest.mark.parametrize("shape", ["1h", "bank"])
def test_every_fft_radix_order_the_tuner_tries(gpu, tmp_path, shape):
    """The autotuner times several orders of the grid's radix passes; every one
    of them, forced through a tuning-cache entry for the shape (method, waves,
    flush period, radix plan, and the small-plan batch this plan keys it by),
    must give the oracle's spectra (n = 60 = 4 3 5 and n = 1200 = 4 4 3 5 5, both ways round,
    sorted, and with the fours split into twos)."""
    from paper_2609_12476_amd import Plan
    say(f"radix orders {shape}")
    if shape == "1h":
        w = synth.semicoherent(hours=0.05, n_mc=2, n_sub=2, seed=19).as_float32_strain()
        n, L = 60, 7680
        orders = [[4, 3, 5], [5, 3, 4], [5, 4, 3], [3, 4, 5], [2, 2, 3, 5]]
    else:
        w = synth.paper_bank(hours=0.05, n_beta=3).as_float32_strain()
        n, L = 1200, 15360
        orders = [[4, 4, 3, 5, 5], [5, 5, 3, 4, 4], [5, 5, 4, 4, 3], [3, 4, 4, 5, 5], [2, 2, 2, 2, 3, 5, 5]]
    Xr, off, ok = oracle.spectra(w)
    for r in orders:
        code = int("".join(str(q) for q in r))
        cache = tmp_path / f"tune_{shape}_{code}.txt"        # the tuner reads each cache path once
        # small plan: the entry is keyed by the shape's valid instances in it
        cache.write_text(f"0 8 {n} {L} 3 1 16 0 1.0 {code} {int(ok.sum())}\n")
        X, _, _, _, cls = run_plan(w, gpu, precision="fp32", tol=1e-6, tune=True, tune_cache=str(cache))
        assert [list(c.radix[:c.n_radix]) for c in cls] == [r] * len(cls), (r, [list(c.radix[:c.n_radix]) for c in cls])
        errs = per_instance_errors(X, Xr, off, ok)
        assert errs.max() <= FP32_SPEC, (r, errs.max())


@pytest.mark.parametrize("flush", [1, 8, 64])
def test_forced_flush_period(gpu, flush):
    say(f"flush period {flush}")
    w = synth.semicoherent(hours=0.05, n_mc=2, n_sub=2, seed=14)
    Xr, off, ok = oracle.spectra(w)
    X, _, _, _, cls = run_plan(w, gpu, precision="fp64", tol=1e-10, flush_period=flush)
    assert cls[0].flush_period == flush
    errs = per_instance_errors(X, Xr, off, ok)
    assert errs.max() <= FP64_SPEC


# ------------------------------------------------------- long phase spans --

@pytest.mark.parametrize("method", ["fused", "cellrun", "staged"])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_heterodyne_phase_beyond_2p31_steps(gpu, method, prec):
    """A band centre of 10 kHz over a 1024 s segment spans about 1e7 cycles of
    the heterodyne phase: 2.6e9 phase-table steps in FP64 (256 per cycle), past
    the 2^31 range of the fused spreaders' table-step conversion, so an FP64
    instance runs on the staged path (phase reduced modulo one cycle) whatever
    method is asked for.  FP32 classes reduce the phase to half a cycle in FP64
    and take its cosine and sine from the hardware, with no such range: they
    keep the method asked for.  Both match the oracle's long-double reduction."""
    say(f"phase beyond 2^31 steps {method} {prec}")
    L, fs = 65536, 64.0
    w = synth.random_small(31, L, 30, 1e-3, f0=50.0, fs=fs, f_lo=10000.0, df=fs / L)
    fc = 10000.0 + 15 * fs / L
    assert fc * L / fs * 256 > 2.0 ** 31
    Xr, off, ok = oracle.spectra(w)
    assert ok[0]
    X, _, valid, _, cls = run_plan(w, gpu, precision=prec, method=method, tol=1e-6)
    assert valid[0] == 1
    expect = {"fused": 2, "cellrun": 3, "staged": 1}[method] if prec == "fp32" else 1
    assert [c.method for c in cls] == [expect]
    e = rel(X, Xr)
    say(f"  rel l2 {e:.3e}")
    assert e <= (FP32_SPEC if prec == "fp32" else 1e-6)


@pytest.mark.parametrize("method", ["fused", "cellrun"])
def test_heterodyne_phase_just_inside_fused_range(gpu, method):
    """Just below 2^30 table steps (about 4e6 cycles at 256 per cycle) the FP64
    fused spreaders keep the instance and match the oracle."""
    say(f"phase inside fused range {method}")
    L, fs = 65536, 64.0
    f_lo = 3600.0                                  # ~3.7e6 cycles over 1024 s: 9.4e8 steps
    w = synth.random_small(32, L, 30, 1e-3, f0=50.0, fs=fs, f_lo=f_lo, df=fs / L)
    steps = (f_lo + 15 * fs / L) * L / fs * 256
    assert 2.0 ** 29 < steps < 2.0 ** 30
    Xr, off, ok = oracle.spectra(w)
    X, _, valid, _, cls = run_plan(w, gpu, precision="fp64", method=method, tol=1e-6)
    assert [c.method for c in cls] == [2 if method == "fused" else 3]
    e = rel(X, Xr)
    say(f"  rel l2 {e:.3e}")
    assert e <= 1e-6


# ------------------------------------------------------------ fused epilogue --

@pytest.mark.parametrize("method,parts", [("cellrun", 1), ("cellrun", 2), ("cellrun", 4), ("fused", 1),
                                          ("fused", 4), ("staged", 2), ("cellrun", 8)])
@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_fused_epilogue_matches_separate_and_oracle(gpu, method, parts, prec):
    """The spreader's own FFT / deconvolution / power (classes of at most four
    waves per instance; asked for explicitly, since this plan is too small for
    the automatic choice) against the separate epilogue kernel and the oracle:
    spectra, power and segment sums."""
    say(f"fused epilogue {method} parts={parts} {prec}")
    w = synth.semicoherent(hours=0.05, n_mc=3, n_sub=3, seed=8)
    tol = 1e-6 if prec == "fp32" else 1e-10
    spec, bound = (FP32_SPEC, FP32_SUM) if prec == "fp32" else (FP64_SPEC, FP64_SPEC)
    kw = dict(precision=prec, tol=tol, method=method, parts=parts)
    Xf, Pf, vf, off, cf = run_plan(w, gpu, epilogue="fused", **kw)
    Xs, Ps, vs, _, cs = run_plan(w, gpu, epilogue="separate", **kw)
    assert [c.epi_fused for c in cf] == [1 if parts <= 4 else 0] * len(cf)
    assert all(c.epi_fused == 0 for c in cs)
    assert np.array_equal(vf, vs)
    ok = vf.astype(bool)
    Xr, offr, okr = oracle.spectra(w)
    assert np.array_equal(okr, vf)
    errs = per_instance_errors(Xf, Xr, off, ok)
    assert errs.max() <= spec, errs.max()
    close = 1e-6 if prec == "fp32" else 1e-13
    assert rel(Xf, Xs) <= close and rel(Pf, Ps) <= close
    assert np.allclose(Pf, np.abs(Xf) ** 2, rtol=1e-5 if prec == "fp32" else 1e-12, atol=0)
    Sf, Uf, soff = run_sum(w, gpu, epilogue="fused", **kw)
    Ss, Us, _ = run_sum(w, gpu, epilogue="separate", **kw)
    Sr, soffr, Ur = oracle.semicoherent(w)
    assert np.array_equal(Uf, Us) and np.array_equal(Uf, Ur)
    for m in range(w.n_tmpl):
        if Ur[m]:
            assert rel(Sf[soff[m]:soff[m + 1]], Sr[soffr[m]:soffr[m + 1]]) <= bound
    assert rel(Sf, Ss) <= close


def test_fused_epilogue_in_grouped_launches(gpu):
    """A ragged batch whose classes of two and four waves per instance run the
    fused epilogue while the classes of eight and sixteen do not, in shared
    grouped launches: every spectrum still matches the oracle."""
    say("fused epilogue in grouped launches")
    w = synth.ragged_batch(n_inst=30, seed=33)
    w.inst_tol = np.where(w.inst_tol < 1e-6, 1e-6, w.inst_tol)
    Xr, off, ok = oracle.spectra(w)
    X, _, valid, off_g, cls = run_plan(w, gpu, precision="fp32", epilogue="fused")
    assert np.array_equal(off, off_g) and np.array_equal(valid, ok)
    fused = {c.epi_fused for c in cls}
    say(f"  {len(cls)} classes, fused flags {sorted(fused)}")
    assert fused == {0, 1}
    for i in range(w.n_inst):
        if ok[i]:
            t = float(w.inst_tol[i])
            assert rel(X[off[i]:off[i + 1]], Xr[off[i]:off[i + 1]]) <= max(t, FP32_SPEC), i


# ------------------------------------------------------------- error paths --

@pytest.mark.parametrize("bad", [float("nan"), float("inf"), -float("inf")])
def test_check_finite_reports_nonfinite_strain(gpu, bad):
    """check_finite scans the strain before any other launch: a NaN or Inf
    anywhere in a segment gives NR_ERR_NONFINITE_INPUT from execute and from
    semicoherent_sum, with the outputs untouched; a finite strain runs."""
    import torch
    from paper_2609_12476_amd import NR_ERR_NONFINITE_INPUT, NrError, Plan
    say(f"check_finite {bad}")
    w = synth.semicoherent(hours=0.02, n_mc=2, n_sub=2, seed=4)
    with Plan.from_workload(w, precision="fp32", check_finite=True) as p:
        x = p.strain_tensor(w.strain, gpu)
        sp, _, valid = p.execute(x)
        torch.cuda.synchronize()
        assert bool(valid.bool().any())
        y = x.clone()
        y[int(w.seg_len[0]) + 17] = bad                  # inside the second segment
        sp2 = torch.full_like(sp, 3.0)
        with pytest.raises(NrError) as e:
            p.execute(y, sp2)
        assert e.value.code == NR_ERR_NONFINITE_INPUT
        stat = torch.full((p.info.stat_bins,), 5.0, dtype=torch.float32, device=gpu)
        with pytest.raises(NrError) as e:
            p.semicoherent_sum(y, None, stat)
        assert e.value.code == NR_ERR_NONFINITE_INPUT
        torch.cuda.synchronize()
        assert bool((sp2 == 3.0).all()) and bool((stat == 5.0).all())


def test_workspace_cap_chunks_then_refuses(gpu):
    """A max_workspace_bytes cap below the grids of the whole plan splits every
    class into chunks (outputs unchanged against the oracle and the uncapped
    plan); a cap below the plan's fixed tables is NR_ERR_OUT_OF_MEMORY at plan
    time."""
    import torch
    from paper_2609_12476_amd import NR_ERR_OUT_OF_MEMORY, NrError, Plan, complex_view
    say("workspace cap")
    w = synth.semicoherent(hours=0.2, n_mc=8, n_sub=20, seed=6)
    X0, _, v0, off, _ = run_plan(w, gpu, precision="fp32")
    S0, U0, soff = run_sum(w, gpu, precision="fp32")
    cap = 3 << 20        # above the two classes' strain copies (1.4 MB) plus one grid chunk, below all grids
    with Plan.from_workload(w, precision="fp32", max_workspace_bytes=cap) as p:
        assert p.info.n_chunks > 1 and p.info.workspace_bytes <= 2 * cap
        x = p.strain_tensor(w.strain, gpu)
        sp, _, valid = p.execute(x)
        stat, used = p.semicoherent_sum(x)
        torch.cuda.synchronize()
        X = complex_view(sp).cpu().numpy().astype(np.complex128)
        S = stat.cpu().numpy().astype(np.float64)
        say(f"  {p.info.n_chunks} chunks, workspace {p.info.workspace_bytes} bytes")
    assert np.array_equal(valid.cpu().numpy(), v0) and np.array_equal(used.cpu().numpy(), U0)
    assert rel(X, X0) <= 1e-6
    for m in range(w.n_tmpl):
        if U0[m]:
            assert rel(S[soff[m]:soff[m + 1]], S0[soff[m]:soff[m + 1]]) <= FP32_SUM
    rng = np.random.default_rng(2)
    idx = np.sort(rng.choice(np.flatnonzero(v0), size=12, replace=False))
    Xr, offr, _ = oracle.spectra(w, inst_idx=idx)
    for j, i in enumerate(idx):
        assert rel(X[off[i]:off[i + 1]], Xr[offr[j]:offr[j + 1]]) <= FP32_SPEC
    with pytest.raises(NrError) as e:
        Plan.from_workload(w, precision="fp32", max_workspace_bytes=64 << 10)
    assert e.value.code == NR_ERR_OUT_OF_MEMORY
