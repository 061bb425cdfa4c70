"""The no-allocation segment sum (nufft_resample_semicoherent_sum_static)
against plan + nufft_resample_semicoherent_sum, through the C ABI.

Two calls in a row (the second with a smaller input, on the scratch the first
one left behind) must each match the allocating entry point to the FP32
segment-sum bound (relative l2 <= 1e-4 per template, counts exact; the same
kernels run, so the sums come out identical in practice), and a plan larger
than the static scratch must be refused with NR_ERR_OUT_OF_MEMORY before any
kernel runs.
"""
import sys

import numpy as np
import pytest

import synth

pytestmark = pytest.mark.gpu

FP32_SUM = 1e-4


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


def _both(w, dev, tol=1e-6, **kw):
    import torch
    from paper_2609_12476_amd import Plan
    from paper_2609_12476_amd import nufft_resample as nr
    with Plan.from_workload(w, tol=tol, precision="fp32", **kw) as p:
        x = p.strain_tensor(w.strain, dev)
        ref, ref_used = p.semicoherent_sum(x)
        torch.cuda.synchronize()
        info = p.info
        segs, tmpls, inst = p._segs, p._tmpls, p._inst
    opt = nr.nufft_resample_default_options()
    opt.precision = nr._PRECISION["fp32"]
    opt.strain_length = len(w.strain)
    for k, v in kw.items():
        setattr(opt, k, v)
    stream = torch.cuda.current_stream()
    opt.stream = nr.c_void_p(stream.cuda_stream)
    stat = torch.zeros(info.stat_bins, dtype=torch.float32, device=dev)
    used = torch.zeros(len(tmpls), dtype=torch.int32, device=dev)
    nr.nufft_resample_semicoherent_sum_static(segs, tmpls, inst, tol, opt, nr.c_void_p(x.data_ptr()), None,
                                              nr.c_void_p(stat.data_ptr()), nr.c_void_p(used.data_ptr()))
    torch.cuda.synchronize()
    return (stat.cpu().numpy().astype(np.float64), used.cpu().numpy(),
            ref.cpu().numpy().astype(np.float64), ref_used.cpu().numpy(), info)


def _compare(w, got, used, ref, ref_used):
    assert np.array_equal(used, ref_used)
    K = int(w.n_bins[0])
    a, b = got.reshape(-1, K), ref.reshape(-1, K)
    worst = 0.0
    for m in range(len(ref_used)):
        if ref_used[m]:
            e = np.linalg.norm(a[m] - b[m]) / np.linalg.norm(b[m])
            worst = max(worst, e)
        else:
            assert not np.any(a[m])
    assert worst <= FP32_SUM, worst
    return worst, bool(np.array_equal(got, ref))


def test_static_sum_matches_allocating_path_twice(gpu):
    say("static-scratch segment sum, two calls")
    w1 = synth.semicoherent(hours=0.1, n_mc=8, n_sub=20, seed=41).as_float32_strain()
    got, used, ref, ref_used, info = _both(w1, gpu)
    say(f"  call 1: {info.n_inst} instances, plan workspace {info.workspace_bytes} bytes")
    worst, same = _compare(w1, got, used, ref, ref_used)
    say(f"  call 1: worst rel l2 {worst:.2e}, bitwise {same}")
    w2 = synth.semicoherent(hours=0.05, n_mc=3, n_sub=5, seed=42).as_float32_strain()
    got, used, ref, ref_used, info = _both(w2, gpu)
    worst, same = _compare(w2, got, used, ref, ref_used)
    say(f"  call 2: {info.n_inst} instances, worst rel l2 {worst:.2e}, bitwise {same}")


def test_static_sum_refuses_plans_beyond_the_scratch(gpu):
    import torch
    from paper_2609_12476_amd import nufft_resample as nr
    say("static-scratch segment sum, oversize plan")
    L = 20_000_000                      # an 80 MB lane-major copy cannot fit 64 MiB
    x = torch.zeros(L, dtype=torch.float32, device=gpu)
    segs = nr.make_segments([0], [L], [256.0], [0.0])
    tmpls = nr.make_templates([0.0], [50.0], [49.5], [1.0 / 30.0], [30], [0.0])
    opt = nr.nufft_resample_default_options()
    opt.strain_length = L
    opt.stream = nr.c_void_p(torch.cuda.current_stream().cuda_stream)
    stat = torch.zeros(30, dtype=torch.float32, device=gpu)
    used = torch.zeros(1, dtype=torch.int32, device=gpu)
    with pytest.raises(nr.NrError) as ei:
        nr.nufft_resample_semicoherent_sum_static(segs, tmpls, None, 1e-6, opt, nr.c_void_p(x.data_ptr()), None,
                                                  nr.c_void_p(stat.data_ptr()), nr.c_void_p(used.data_ptr()))
    assert ei.value.code == nr.NR_ERR_OUT_OF_MEMORY and "static scratch" in str(ei.value)
    torch.cuda.synchronize()
    assert not torch.any(stat) and int(used[0]) == 0
    # options that would allocate are refused
    opt.use_graph = 1
    with pytest.raises(nr.NrError) as ei:
        nr.nufft_resample_semicoherent_sum_static(segs, tmpls, None, 1e-6, opt, nr.c_void_p(x.data_ptr()), None,
                                                  nr.c_void_p(stat.data_ptr()), nr.c_void_p(used.data_ptr()))
    assert ei.value.code == nr.NR_ERR_INVALID_ARG
