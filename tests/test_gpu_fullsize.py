"""Parity at the full benchmark sizes, in the launch configuration bench.py
times (fused FP32, tol 1e-6), on outputs the oracle computes one by one:
sampled instances of the 1 h / 153,600-instance workload and segment sums of
sampled templates, plus the full 512-instance ragged batch sampled."""
import sys

import numpy as np
import pytest

import oracle
import synth

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def rel(a, b):
    return np.linalg.norm(a - b) / np.linalg.norm(b)


@pytest.mark.parametrize("method", ["fused", "cellrun"])
def test_semicoherent_1h_sampled(gpu, method):
    say(f"full-size 1 h workload, sampled, {method}")
    import torch
    from paper_2609_12476_amd import Plan, complex_view
    w = synth.semicoherent(hours=1.0, n_mc=64, n_sub=20, seed=1).as_float32_strain()
    with Plan.from_workload(w, tol=1e-6, precision="fp32", method=method) as p:
        assert p.info.n_inst == 153600
        x = p.strain_tensor(w.strain, gpu)
        sp, _, valid = p.execute(x, want=("spectra", "valid"))
        stat, used = p.semicoherent_sum(x)
        torch.cuda.synchronize()
        X = complex_view(sp).cpu().numpy().astype(np.complex128)
        ok = valid.cpu().numpy().astype(bool)
        boff = p.bin_offsets()
        S = stat.cpu().numpy().astype(np.float64)
        U = used.cpu().numpy()
        soff = p.stat_offsets()
    rng = np.random.default_rng(17)
    idx = np.sort(rng.choice(np.flatnonzero(ok), size=48, replace=False))
    Xr, off, okr = oracle.spectra(w, inst_idx=idx)
    assert okr.all()
    errs = [rel(X[boff[i]:boff[i + 1]], Xr[off[j]:off[j + 1]]) for j, i in enumerate(idx)]
    say(f"  spectra: max rel {max(errs):.2e}")
    assert max(errs) <= 1e-5
    # validity flags of every instance against the oracle's rule
    s_all, m_all = w.instances()
    for i in rng.choice(w.n_inst, size=2000, replace=False):
        s, m = s_all[i], m_all[i]
        assert ok[i] == oracle.valid(w.mc[m], w.f0[m], w.f_max[m], w.seg_t[s], w.seg_fs[s], w.seg_len[s])
    # segment sums of sampled templates (all 120 segments each)
    tm = np.sort(rng.choice(w.n_tmpl, size=8, replace=False))
    sub = synth.Workload(**{**w.__dict__, "mc": w.mc[tm], "f0": w.f0[tm], "f_lo": w.f_lo[tm],
                            "df": w.df[tm], "n_bins": w.n_bins[tm], "f_max": w.f_max[tm]})
    Sr, soff_r, used_r = oracle.semicoherent(sub)
    for q, m in enumerate(tm):
        assert U[m] == used_r[q]
        if used_r[q]:
            e = rel(S[soff[m]:soff[m + 1]], Sr[soff_r[q]:soff_r[q + 1]])
            assert e <= 1e-4, (m, e)


def test_ragged_512_sampled(gpu):
    say("full ragged batch, sampled")
    import torch
    from paper_2609_12476_amd import Plan, complex_view
    w = synth.ragged_batch(n_inst=512, seed=2)
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with Plan.from_workload(w, precision="auto", use_graph=True, stream=s) as p:
            x = p.strain_tensor(w.strain, gpu)
            sp, _, valid = p.execute(x, want=("spectra", "valid"))
            sp2, _, _ = p.execute(x, want=("spectra",))      # graph replay
            s.synchronize()
            assert torch.equal(sp, sp2)
            X = complex_view(sp).cpu().numpy().astype(np.complex128)
            ok = valid.cpu().numpy().astype(bool)
            boff = p.bin_offsets()
    rng = np.random.default_rng(19)
    idx = np.sort(rng.choice(np.flatnonzero(ok), size=24, replace=False))
    Xr, off, _ = oracle.spectra(w, inst_idx=idx)
    for j, i in enumerate(idx):
        t = w.inst_tol[i]
        bound = max(t, 1e-5) if t >= 1e-6 else max(t, 1e-11)
        assert rel(X[boff[i]:boff[i + 1]], Xr[off[j]:off[j + 1]]) <= bound, (i, t)


def test_full_sweep_6h_sampled_sums(gpu):
    """The 6 h sweep (720 segments x 2048 chirp masses x 20 sub-bands =
    29,491,200 instances, chunked) in the configuration bench.py times: the
    segment sums and counts of sampled templates against the oracle."""
    import torch
    from paper_2609_12476_amd import Plan
    say("full sweep 6 h, sampled templates")
    w = synth.semicoherent(hours=6.0, n_mc=2048, n_sub=20, seed=3, tol=1e-6).as_float32_strain()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        with Plan.from_workload(w, precision="fp32", tol=1e-6, use_graph=True, stream=s) as p:
            assert p.info.n_inst == 29491200
            x = p.strain_tensor(w.strain, gpu)
            stat, used = p.semicoherent_sum(x)
            s.synchronize()
            S = stat.cpu().numpy().astype(np.float64)
            U = used.cpu().numpy()
            soff = p.stat_offsets()
    rng = np.random.default_rng(29)
    tm = np.sort(rng.choice(np.flatnonzero(U > 0), size=4, replace=False))
    sub = synth.Workload(**{**w.__dict__, "mc": w.mc[tm], "f0": w.f0[tm], "f_lo": w.f_lo[tm],
                            "df": w.df[tm], "n_bins": w.n_bins[tm], "f_max": w.f_max[tm]})
    Sr, soff_r, used_r = oracle.semicoherent(sub)
    for q, m in enumerate(tm):
        assert U[m] == used_r[q]
        e = rel(S[soff[m]:soff[m + 1]], Sr[soff_r[q]:soff_r[q + 1]])
        say(f"  template {m}: {U[m]} segments, rel l2 {e:.2e}")
        assert e <= 1e-4, (m, e)


@pytest.mark.parametrize("method", ["auto", "fused"])
def test_paper_beta_bank_sampled(gpu, method):
    """The paper's own coherent workload (Sec. III.A, VI): 1 h at 512 Hz in 120
    segments of 30 s, each resampled from its own start with the 69 beta
    templates uniform over [3e-8, 7e-4] and transformed onto the 600 bins of
    40-60 Hz, in the launch configuration bench.py times (FP32, tol 1e-6; the
    automatic method takes cell runs with four waves per instance).  48 sampled
    spectra against the oracle, each <= 1e-5 relative l2; every spectrum of the
    bank is valid (no frequency cut)."""
    say(f"paper beta bank, sampled, {method}")
    import torch
    from paper_2609_12476_amd import Plan, complex_view
    w = synth.paper_bank(hours=1.0).as_float32_strain()
    with Plan.from_workload(w, tol=1e-6, precision="fp32", method=method) as p:
        assert p.info.n_inst == 120 * 69 and p.info.n_valid == p.info.n_inst
        cls = p.classes()
        say(f"  classes {[(c.w, c.n, c.degree, c.parts, c.method) for c in cls]}")
        if method == "auto":
            assert all(c.method == 3 for c in cls)
        x = p.strain_tensor(w.strain, gpu)
        sp, pw, valid = p.execute(x)
        torch.cuda.synchronize()
        X = complex_view(sp).cpu().numpy().astype(np.complex128)
        P = pw.cpu().numpy().astype(np.float64)
        boff = p.bin_offsets()
    rng = np.random.default_rng(23)
    idx = np.sort(rng.choice(w.n_inst, size=48, replace=False))
    Xr, off, okr = oracle.spectra(w, inst_idx=idx)
    assert okr.all()
    errs = [rel(X[boff[i]:boff[i + 1]], Xr[off[j]:off[j + 1]]) for j, i in enumerate(idx)]
    say(f"  spectra: max rel {max(errs):.2e}, median {np.median(errs):.2e}")
    assert max(errs) <= 1e-5
    assert np.allclose(P, np.abs(X) ** 2, rtol=1e-5, atol=0)
