#!/usr/bin/env python3
"""Throughput of batched semicoherent NUFFT resampling on one MI355X.

One step = one semicoherent sum over the whole workload: for every
(segment, template) instance the resampled times, the spreading, the FFT,
the deconvolution, the power and the per-template segment sum, all in the
gfx950 kernels (FP64 tau and phase reduction, FP32 spreading/FFT/power).

Workload (default): 1 h of 256 Hz white Gaussian noise with one injected
0PN chirp, split into 120 segments of 30 s; 64 chirp-mass templates
log-spaced over [5e-4, 1e-1] Msun x 20 sub-bands of 1 Hz over 40-60 Hz;
spreading tolerance 1e-6, 2x upsampled grid: 153,600 instances.

Prints one JSON line.  Outside the timed region it also
  - checks the FP32 spectra of every instance against the FP64 path
    (tolerance 1e-10) and the summed statistic,
  - times the plain FP64 path (same kernels, FP64 class, same tolerance),
  - times the oracle on a bounded seeded sample of instances on the host
    cores and checks the GPU spectra of that sample against it.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = ("segment×template spectra/s at ≤1e-5 rel err vs FP64 plain; "
          "spread+FFT HBM GB/s")
HBM_PEAK_GBS = 8000.0
# VALU lane-operations per second: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz
# (one FP32 or FP64 FMA per lane per cycle without packed FP32).
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
METHOD_NAME = {1: "staged", 2: "fused", 3: "cellrun"}


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--method", default="auto", choices=["auto", "fused", "staged", "cellrun"])
    ap.add_argument("--hours", type=float, default=1.0)
    ap.add_argument("--n-mc", type=int, default=64)
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-direct", action="store_true", help="skip the GPU direct-sum baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-check", action="store_true")
    ap.add_argument("--no-extra", action="store_true", help="skip the beta-bank and ragged-512 keys")
    ap.add_argument("--cpu-sample", type=int, default=3072,
                    help="instances timed on the oracle (seeded sample)")
    ap.add_argument("--copy-mib", type=int, default=256,
                    help="size of the plain copy kernel run once for counter calibration")
    ap.add_argument("--workload", default="semicoherent_1h",
                    choices=["semicoherent_1h", "full_sweep_6h", "ragged_512", "paper_beta_bank", "stackslide_1h",
                             "strobo_vs_nufft"],
                    help="semicoherent_1h is the headline; the others print their own line")
    ap.add_argument("--tune", action="store_true", help="autotune the spreader per shape")
    ap.add_argument("--moment-mode", type=int, default=0, help="0 auto, 1 per cell, 2 cumulative")
    ap.add_argument("--flush-period", type=int, default=0)
    return ap.parse_args()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def committed_counter(kernel_key, field="traffic_bytes_per_launch"):
    """A per-launch figure of kernel_key recorded as `field[kernel]: value` in
    the rocprofv3 summaries under profiles/, or None when none records it or
    the kernel sources named there changed since it was measured."""
    import glob
    import hashlib
    import re
    for path in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.md"))):
        txt = open(path).read()
        h = re.search(r"^source_sha256: ([0-9a-f]+)", txt, re.M)
        src = re.search(r"^sources: (.+)", txt, re.M)
        val = None
        for m in re.finditer(re.escape(field) + r"\[(.+?)\]: (\d+)", txt):
            if m.group(1) == kernel_key:
                val = float(m.group(2))
        if val is None or not (h and src):
            continue
        digest = hashlib.sha256()
        for rel in src.group(1).split():
            with open(os.path.join(ROOT, rel), "rb") as f:
                digest.update(f.read())
        if digest.hexdigest() == h.group(1):
            return val
    return None


def committed_traffic(kernel_key):
    """HBM bytes per launch of kernel_key (FETCH_SIZE and WRITE_SIZE scaled by
    the copy-kernel calibration) from the rocprofv3 summaries under profiles/,
    or None when none covers it or its kernel sources changed since."""
    return committed_counter(kernel_key, "traffic_bytes_per_launch")


def algorithmic_ops(classes):
    """VALU lane-operations the fused spreader needs, by the per-sample op model:
    tau series (degree + 1 FMAs; 40 for the log1p/expm1 form) + 6 for the two
    products and reductions mod 1, 2 to split the grid position, 13 for the
    sin/cos pair, 2 for the heterodyne product and 3D + 1 for the Chebyshev
    moments of degree D."""
    tot = 0
    for c in classes:
        series = c.series_terms + (c.n_points - c.fallback_points) + 40 * c.fallback_points
        tot += series + c.n_points * (6 + 2 + 13 + 2 + 3 * c.degree + 1)
    return tot


def spread_fft_bytes(classes, strain_bytes, stat_bins, K):
    """Algorithmic HBM bytes of the spread, FFT and segment-sum stages of one
    step: the strain once, the point stream of staged classes (read by the
    spreader), the grids of classes whose FFT runs in a second kernel (written
    and read back), the power rows (written, then read by the row sums) and
    the statistic."""
    b = strain_bytes + stat_bins * 4
    for c in classes:
        csize = 16 if c.fp64 else 8
        if c.method == 1:                                    # NR_METHOD_STAGED
            b += c.n_points * csize
        if not c.epi_fused:
            b += 2 * c.n_inst * c.n * csize
        b += 2 * c.n_inst * K * 4
    return b


def time_steps(plan, x, stat, used, steps, warmup):
    import torch
    for _ in range(warmup):
        stat.zero_()
        used.zero_()
        plan.semicoherent_sum(x, None, stat, used)
    torch.cuda.synchronize()
    plan.stage_times()  # reset the per-stage accumulation
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        stat.zero_()
        used.zero_()
        plan.semicoherent_sum(x, None, stat, used)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    return t1 - t0, plan.stage_times()


def measure_workload(args, dev, workload, steps, check=16, tune=False, method="auto"):
    """Time one of the secondary workloads (HIP-graph replay), its spreader's
    VALU fraction by the op model (a second, profiled plan) and a sampled
    oracle check; returns the result dict."""
    import torch

    import oracle
    import synth
    from paper_2609_12476_amd import Plan, complex_view

    stream = torch.cuda.Stream()
    out = {}
    with torch.cuda.stream(stream):
        if workload == "ragged_512":
            w = synth.ragged_batch(n_inst=512, seed=2)
            kw = dict(precision="auto", tune=tune, method=method)
            mode = "execute"
        elif workload == "paper_beta_bank":
            w = synth.paper_bank(hours=1.0).as_float32_strain()
            kw = dict(precision="fp32", tol=1e-6, tune=tune, method=method)
            mode = "execute"
        else:
            w = synth.semicoherent(hours=6.0, n_mc=2048, n_sub=20, seed=3, tol=1e-6).as_float32_strain()
            kw = dict(precision="fp32", tol=1e-6, tune=tune, method=method)
            mode = "sum"
        kw.update(flush_period=args.flush_period, moment_mode=args.moment_mode)
        log(f"{w.name}: planning {w.n_inst} instances")
        t0 = time.perf_counter()
        plan = Plan.from_workload(w, stream=stream, use_graph=True, **kw)
        plan_s = time.perf_counter() - t0
        x = plan.strain_tensor(w.strain, dev)
        info = plan.info

        def stepper(pl):
            if mode == "execute":
                sp = torch.empty(2 * info.total_bins, dtype=pl.out_dtype, device=dev)
                pw = torch.empty(info.total_bins, dtype=pl.out_dtype, device=dev)
                va = torch.empty(pl.n_inst, dtype=torch.uint8, device=dev)
                return lambda: pl.execute(x, sp, pw, va)
            st = torch.zeros(info.stat_bins, dtype=pl.out_dtype, device=dev)
            us = torch.zeros(pl.n_tmpls, dtype=torch.int32, device=dev)
            return lambda: pl.semicoherent_sum(x, None, st, us)

        step = stepper(plan)
        for _ in range(args.warmup):
            step()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        el = time.perf_counter() - t0
        cls = plan.classes()
        samples = int(sum(c.n_points for c in cls))
        out.update({"metric": f"{w.name} spectra/s", "value": info.n_valid * steps / el,
                    "ms_per_step": el / steps * 1e3, "steps": steps, "samples_per_s": samples * steps / el,
                    "config": {"workload": w.name, "instances": int(info.n_inst), "valid": int(info.n_valid),
                               "samples": samples, "classes": len(cls), "chunks": int(info.n_chunks),
                               "graph": True, "tuned": bool(tune), "plan_seconds": plan_s},
                    "class_shapes": [(c.fp64, c.w, c.n, c.degree, c.parts, c.method, c.flush_period, c.n_inst)
                                     for c in cls]})
        # spreader time and VALU fraction from a profiled plan of the same workload
        prof = Plan.from_workload(w, stream=stream, profile=True, **kw)
        pstep = stepper(prof)
        pstep()
        torch.cuda.synchronize()
        prof.stage_times()
        for _ in range(steps):
            pstep()
        stt = prof.stage_times()
        spread_ms = stt["spread"][0] / steps
        if all(c.method in (2, 3) for c in cls):
            ops = algorithmic_ops(cls)
            out["spread_ms_per_step"] = spread_ms
            out["spread_valu_frac"] = ops / (spread_ms * 1e-3) / 1e12 / VALU_PEAK_TOPS
            # executed VALU instructions of the one spread launch per step, as
            # recorded per workload in the committed rocprofv3 summary
            if len(cls) == 1 and cls[0].method == 3 and not cls[0].fp64:
                key = f"{workload}:nr::spread_runs_kernel<float, {cls[0].degree}, false>"
                vi = committed_counter(key, "valu_instructions_per_launch")
                if vi is not None:
                    out["spread_valu_issue_frac_counters"] = vi * 4 / (1024 * 2.4e9 * spread_ms * 1e-3)
            out["spread_valu_basis"] = "per-sample op model (algorithmic_ops) over the summed spread launches"
        out["stage_ms_per_step"] = {k: v[0] / steps for k, v in stt.items()}
        prof.close()
        # sampled parity against the oracle
        if check:
            rng = np.random.default_rng(7)
            ok = plan.valid_mask().astype(bool)
            idx = np.sort(rng.choice(np.flatnonzero(ok), size=min(check, int(ok.sum())), replace=False))
            sp2, _, _ = plan.execute(x, want=("spectra",))
            torch.cuda.synchronize()
            X = complex_view(sp2).cpu().numpy().astype(np.complex128)
            Xr, off, _ = oracle.spectra(w, inst_idx=idx)
            boff = plan.bin_offsets()
            errs = [np.linalg.norm(X[boff[i]:boff[i + 1]] - Xr[off[j]:off[j + 1]]) /
                    np.linalg.norm(Xr[off[j]:off[j + 1]]) for j, i in enumerate(idx)]
            out["oracle_check"] = {"instances": len(idx), "spectra_rel_l2_max": float(np.max(errs))}
        plan.close()
    return out


def mlp_step_timing(dev, B=1024, steps=200):
    """One training step of the proposal's network (forward, backward, Adam) on a
    batch of B rows: HIP-event time per step and the dense-product throughput of
    its two hidden layers (forward, da1 and the two weight gradients)."""
    import torch

    import synth
    from paper_2609_12476_amd.mlp import Mlp
    g = torch.Generator(device=dev).manual_seed(5)
    x = torch.randn(B, 64, generator=g, device=dev)
    y = (torch.rand(B, generator=g, device=dev) < 0.5).float()
    net = Mlp(max_batch=B, params=synth.mlp_init_params(5))
    for _ in range(10):
        net.train_step(x, y, 1e-3)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(steps):
        net.train_step(x, y, 1e-3)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) / steps * 1e3
    net.close()
    # dense flops per step: forward 2B(64*256 + 256*256), da1 2B*256*256, dW1 2B*64*256, dW2 2B*256*256
    flops = 2.0 * B * (64 * 256 + 256 * 256) + 2.0 * B * 256 * 256 + 2.0 * B * (64 * 256 + 256 * 256)
    return {"batch": B, "us_per_step": us, "dense_tflops": flops / (us * 1e-6) / 1e12,
            "peak_fp32_mfma_tflops": 157.3}


def other_workload(args, dev):
    """Throughput of the non-headline workloads (one JSON line each)."""
    steps = max(2, args.steps // (10 if args.workload == "full_sweep_6h" else 1))
    out = {"unit": "spectra/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic",
           "warmup": args.warmup}
    out.update(measure_workload(args, dev, args.workload, steps, tune=args.tune, method=args.method))
    print(json.dumps(out), flush=True)


def stackslide_workload(args, dev):
    """Weighted stack-slide along 0PN tracks over the paper's 1 h spectra
    (120 segments x 69 beta x 600 bins from the NUFFT path): 2048 chirp masses
    log-spaced over [5e-4, 1e-1] Msun x 120 x 8 start times (1.97e6 tracks)."""
    import torch

    import synth
    from oracle import stackslide as oss
    from paper_2609_12476_amd import Plan
    from paper_2609_12476_amd import stackslide as ss

    w = synth.paper_bank(hours=1.0).as_float32_strain()
    n_seg, K, L = w.n_seg, int(w.n_bins[0]), int(w.seg_len[0])
    betas, _ = synth.beta_bank(69)
    log(f"spectra: {w.n_inst} instances")
    with Plan.from_workload(w, precision="fp32", tol=1e-6) as pl:
        x = pl.strain_tensor(w.strain, dev)
        _, power, _ = pl.execute(x, want=("power",))
    power_t = ss.nr_ss_transpose(power, len(betas), n_seg, K)
    torch.cuda.synchronize()
    copy_calibration(args, dev)
    mcs = synth.log_spaced_mc(2048)
    S = 8
    out = {"unit": "tracks/s", "n_gpus": 1, "higher_is_better": True, "data": "synthetic", "dtype": "f32"}
    res = {}
    for layout, P in ((0, power), (1, power_t)):
        g = ss.geometry(n_seg, len(betas), K, 30.0, 40.0, 1.0 / 30.0, 40.0, 60.0, 2.0 / L, layout=layout)
        with ss.StackSlide(g, betas, mcs, S) as p:
            ns, used = p.execute(P)
            torch.cuda.synchronize()
            for _ in range(args.warmup):
                p.execute(P, ns, used)
            torch.cuda.synchronize()
            ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            ev0.record()
            for _ in range(args.steps):
                p.execute(P, ns, used)
            ev1.record()
            torch.cuda.synchronize()
            ms = ev0.elapsed_time(ev1) / args.steps
            reads = int(used.to(torch.int64).sum().item())
            res[layout] = (ms, reads, ns.cpu().numpy(), p.n_tracks)
    ms, reads, ns, n_tracks = res[1]
    alg_bytes = reads * 4 + n_tracks * 8       # one power value per (track, segment); n_sigma and count out
    gbs = alg_bytes / (ms * 1e-3) / 1e9
    out.update({"metric": "stack-slide tracks/s (paper 1 h spectra)", "value": n_tracks / (ms * 1e-3),
                "ms_per_step": ms, "steps": args.steps, "warmup": args.warmup,
                "config": {"workload": "stackslide_1h_120seg_69beta_600bins_2048mc_x8t0", "tracks": n_tracks,
                           "power_reads": reads, "layout": "[beta][bin][segment]"},
                "layout0_ms": res[0][0],
                "roofline": {"kernel": "gather_kernel<1, false>", "bound": "hbm", "achieved": gbs,
                             "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": gbs / HBM_PEAK_GBS,
                             "traffic": committed_traffic("gather_kernel<1, false>"),
                             "traffic_unit": "bytes per launch", "avg_launch_ms": ms,
                             "note": "the 19.9 MB of spectra stay in the L2/MALL caches across tracks"}})
    # sampled parity and the oracle's rate on the host
    P = power.cpu().numpy().astype(np.float64).reshape(len(betas), n_seg, K)
    rng = np.random.default_rng(11)
    cand = [(int(c), int(q) // S, int(q) % S) for c, q in
            zip(rng.integers(0, len(mcs), 256), rng.integers(0, n_seg * S, 256))]
    t0 = time.perf_counter()
    ref, _ = oss.n_sigma(P, mcs, S, 30.0, betas, 40.0, 1.0 / 30.0, 40.0, 60.0, 2.0 / L, tracks=cand)
    cpu_s = time.perf_counter() - t0
    err = max(abs(float(ns[c, i0 * S + s]) - ref[c, i0 * S + s]) for (c, i0, s) in cand)
    out["oracle_check"] = {"tracks": len(cand), "n_sigma_abs_err_max": err,
                           "layout0_vs_layout1_max": float(np.abs(res[0][2] - ns).max())}
    out["cpu_baseline"] = {"value": len(cand) / cpu_s, "unit": "tracks/s", "cores": 1, "kind": "oracle",
                           "sample": f"{len(cand)} seeded tracks of the {n_tracks} (pure-Python FP64 loop)"}
    print(json.dumps(out))
    return out


def copy_calibration(args, dev, reps=5):
    """Plain device copies of known size (the memory counters of one are the
    calibration of FETCH_SIZE / WRITE_SIZE); returns the measured copy rate in
    GB/s (read + write bytes over the median HIP-event time), or None."""
    import torch
    if args.copy_mib <= 0:
        return None
    a = torch.ones(args.copy_mib << 18, dtype=torch.float32, device=dev)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    ms = []
    for _ in range(reps):
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        b.copy_(a)
        e1.record()
        torch.cuda.synchronize()
        ms.append(e0.elapsed_time(e1))
    del a, b
    return 2.0 * (args.copy_mib << 20) / (float(np.median(ms)) * 1e-3) / 1e9


def host_cpu():
    """Model string and usable core count of the host."""
    model = None
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except AttributeError:
        usable = os.cpu_count()
    return {"model": model, "logical_cpus": os.cpu_count(), "usable_cpus": usable}


def _median_ms(fn, reps=5):
    import torch
    fn()
    torch.cuda.synchronize()
    out = []
    for _ in range(reps):
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        fn()
        b.record()
        torch.cuda.synchronize()
        out.append(a.elapsed_time(b))
    return float(np.median(out))


def strobo_workload(args, dev):
    """NUFFT vs stroboscopic resampling at equal accuracy, the comparison of the
    paper's NUFFT speed-up figure: f0 = 20 Hz, Mc = 1e-2 Msun, resampled series
    at 512 Hz, T_coh = 32, 256 and 2048 s, with 2^22 samples of data in each
    case (256, 32 and 4 segments, each its own time reference) so that both
    methods run batched.  The input is an analytic chirp with no noise, so each
    method's error is its relative l2 distance, over the 64 bins around 20 Hz
    of segment 0, from its own exact value: the direct non-uniform sum (the
    oracle) for the NUFFT, the tau-uniform tone for the stroboscopic method.
    The stroboscopic FFT yields the whole 0-256 Hz band by construction; the
    NUFFT is timed for the whole band (256 sub-band templates of 1 Hz) and for
    a 20 Hz band (10-30 Hz, 20 sub-bands), the width of the paper's search."""
    import torch

    import oracle
    import synth
    from oracle import strobo as ost
    from paper_2609_12476_amd import Plan, complex_view, strobo

    f0, mc, fs, phi0 = 20.0, 1e-2, 512.0, 0.3
    total = 1 << 22
    table = []
    for T, o_max in ((32.0, 128), (256.0, 64), (2048.0, 8)):
        L = int(T * fs)
        n_seg = total // L
        df = 1.0 / T
        Kt = int(round(T))
        t = np.arange(L) / fs
        x1 = 0.5 * np.exp(1j * synth.chirp_phase(t, f0, mc, 0.0, phi0))
        x = np.tile(x1, n_seg)
        lo = 20.0 - 32 * df                        # the 64 evaluation bins: 20 Hz - 32 df ...
        ref = oracle.spectrum(x1, fs, 0.0, mc, f0, lo, df, 64)[0]
        row = {"t_coh": T, "segments": n_seg}
        for band, (b0, nb) in (("full", (0, 256)), ("band20", (10, 20))):
            w = synth.Workload(name=f"strobo_cmp_{T:g}s", strain=x,
                               seg_offset=np.arange(n_seg, dtype=np.int64) * L,
                               seg_len=np.full(n_seg, L, np.int64), seg_fs=np.full(n_seg, fs),
                               seg_t=np.zeros(n_seg), mc=np.full(nb, mc), f0=np.full(nb, f0),
                               f_lo=np.arange(b0, b0 + nb, dtype=np.float64), df=np.full(nb, df),
                               n_bins=np.full(nb, Kt, np.int32), f_max=np.zeros(nb))
            res = []
            for tol, prec in ((1e-1, "fp32"), (1e-2, "fp32"), (1e-3, "fp32"), (1e-4, "fp32"), (1e-6, "fp32"),
                              (1e-9, "fp64")):
                try:
                    p = Plan.from_workload(w, tol=tol, precision=prec)
                except Exception as e:             # e.g. an FP64 grid beyond the LDS limit
                    res.append({"tol": tol, "precision": prec, "unsupported": str(e)[:120]})
                    continue
                with p:
                    xs = p.strain_tensor(x, dev)
                    sp = torch.empty(2 * p.info.total_bins, dtype=p.out_dtype, device=dev)
                    ms = _median_ms(lambda: p.execute(xs, sp, None, None))
                    X = complex_view(sp).cpu().numpy().astype(np.complex128)
                    off = p.bin_offsets()                      # instance = template * n_seg + segment
                    i19, i20 = (19 - b0) * n_seg, (20 - b0) * n_seg
                    got = np.concatenate([X[off[i19] + Kt - 32:off[i19 + 1]], X[off[i20]:off[i20] + 32]])
                res.append({"tol": tol, "precision": prec, "ms": ms,
                            "err": float(np.linalg.norm(got - ref) / np.linalg.norm(ref))})
                log(f"T={T:g} {band} nufft tol {tol:g}: {ms:.3f} ms err {res[-1]['err']:.2e}")
            row["nufft_" + band] = res
        strob = []
        O = 1
        while O <= o_max:
            fs_o = fs * O
            n = L * O
            seg = torch.from_numpy((0.5 * np.exp(1j * synth.chirp_phase(np.arange(n) / fs_o, f0, mc, 0.0, phi0)))
                                   .astype(np.complex64)).to(dev)
            xo = seg.repeat(n_seg)
            del seg
            ms = _median_ms(lambda: strobo.spectrum(xo, fs_o, O, mc, f0, 0.0, df, 256 * Kt, n_seg=n_seg))
            S = strobo.spectrum(xo, fs_o, O, mc, f0, lo, df, 64, n_seg=n_seg)[0].cpu().numpy().astype(np.complex128)
            M = strobo.nr_strobo_points(fs_o, n, mc, f0)
            lim = ost.tone_limit(0.5, phi0, f0, M, fs_o, O, lo, df, 64)
            strob.append({"oversample": O, "ms": ms, "err": float(np.linalg.norm(S - lim) / np.linalg.norm(lim))})
            log(f"T={T:g} strobo O={O}: {ms:.3f} ms err {strob[-1]['err']:.2e}")
            del xo
            torch.cuda.empty_cache()
            O *= 2
        row["stroboscopic"] = strob
        for band in ("full", "band20"):
            speed = {}
            for eps in (0.025, 1e-2, 1e-3):
                tn = min([r["ms"] for r in row["nufft_" + band] if r.get("err", 1.0) <= eps], default=None)
                ts = min([r["ms"] for r in strob if r["err"] <= eps], default=None)
                speed[f"{eps:g}"] = (ts / tn) if (tn and ts) else None
            row["speedup_" + band] = speed
        table.append(row)
    out = {"metric": "stroboscopic / NUFFT time at resampling error 0.025 (T_coh 256 s, 20 Hz band)",
           "value": table[1]["speedup_band20"]["0.025"], "unit": "x", "higher_is_better": True, "n_gpus": 1,
           "data": "synthetic",
           "config": {"workload": "strobo_vs_nufft_f0_20Hz_mc_1e-2_512Hz", "t_coh": [r["t_coh"] for r in table],
                      "samples": total},
           "table": table}
    print(json.dumps(out))
    return out


def main():
    args = parse()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on exactly one GPU: there is no multi-GPU path (instances are "
              "independent; several GPUs would each take a share of the templates).", file=sys.stderr)
        sys.exit(2)

    import torch

    import synth
    from paper_2609_12476_amd import Plan, complex_view

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda:0")
    if args.workload == "stackslide_1h":
        return stackslide_workload(args, dev)
    if args.workload == "strobo_vs_nufft":
        return strobo_workload(args, dev)
    if args.workload != "semicoherent_1h":
        return other_workload(args, dev)
    log("generating workload")
    w = synth.semicoherent(hours=args.hours, n_mc=args.n_mc, n_sub=20, seed=1, tol=1e-6)
    w32 = w.as_float32_strain()           # the FP32 path's input values; the FP64 runs use the same
    plan = Plan.from_workload(w32, tol=1e-6, precision="fp32", method=args.method, profile=True,
                              moment_mode=args.moment_mode, flush_period=args.flush_period, tune=args.tune)
    info = plan.info
    cls = plan.classes()
    x32 = plan.strain_tensor(w32.strain, dev)
    stat = torch.zeros(info.stat_bins, dtype=torch.float32, device=dev)
    used = torch.zeros(plan.n_tmpls, dtype=torch.int32, device=dev)
    log(f"plan: {info.n_inst} instances, {info.n_valid} valid, classes "
        f"{[(c.fp64, c.w, c.n, c.degree, c.parts) for c in cls]}, chunks {info.n_chunks}")

    # accuracy: FP32 vs the FP64 path on every instance (before the timed
    # steps: outside the timed region, and the GPU's clocks settle meanwhile)
    accuracy = None
    if not args.no_check:
        log("accuracy check vs fp64")
        sp32, _, valid = plan.execute(x32, want=("spectra", "valid"))
        p64 = Plan.from_workload(w32, tol=1e-10, precision="fp64", method=args.method)
        x64 = p64.strain_tensor(w32.strain, dev)
        sp64, _, _ = p64.execute(x64, want=("spectra",))
        s64, u64 = p64.semicoherent_sum(x64)
        stat.zero_(); used.zero_()
        plan.semicoherent_sum(x32, None, stat, used)
        torch.cuda.synchronize()
        K = 30
        a = complex_view(sp32).to(torch.complex128).view(-1, K)
        b = complex_view(sp64).view(-1, K)
        v = valid.bool()
        num = torch.linalg.vector_norm(a - b, dim=1)[v]
        den = torch.linalg.vector_norm(b, dim=1)[v]
        e = (num / den).cpu().numpy()
        sa = stat.double().view(-1, K)
        sb = s64.view(-1, K)
        keep = u64 > 0
        es = (torch.linalg.vector_norm(sa - sb, dim=1)[keep] /
              torch.linalg.vector_norm(sb, dim=1)[keep]).cpu().numpy()
        accuracy = {"spectra_rel_l2_max": float(e.max()), "spectra_rel_l2_median": float(np.median(e)),
                    "stat_rel_l2_max": float(es.max()), "reference": "gpu fp64 path, tol 1e-10",
                    "n_used_equal": bool(torch.equal(used, u64))}
        del sp32, sp64, a, b, p64, x64
        torch.cuda.empty_cache()

    copy_gbs = copy_calibration(args, dev)

    log("timing fp32")
    el, st = time_steps(plan, x32, stat, used, args.steps, args.warmup)
    ms_step = el / args.steps * 1e3
    value = info.n_valid * args.steps / el
    out = {
        "metric": METRIC, "value": value, "unit": "spectra/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"semicoherent_{args.hours:g}h_{w.n_seg}seg_{args.n_mc}mc_x20subbands_256Hz",
                   "instances": int(info.n_inst), "valid_instances": int(info.n_valid),
                   "samples_per_segment": int(w.seg_len[0]), "bins_per_spectrum": 30,
                   "tol": 1e-6, "sigma": 2.0, "method": args.method,
                   "spreaders": sorted({METHOD_NAME[c.method] for c in cls}), "kernel_width": cls[0].w,
                   "grid": cls[0].n, "degree": cls[0].degree, "parallelism": "single_gpu"},
        "all_instance_rate": info.n_inst * args.steps / el,
        "copy_gbs": copy_gbs,
        "host_cpu": host_cpu(),
    }
    stage_ms = {k: v[0] / args.steps for k, v in st.items()}
    out["stage_ms_per_step"] = stage_ms

    # roofline of the dominant kernel
    dom = max(("tau", "spread", "epilogue"), key=lambda k: stage_ms[k])
    launches = st[dom][1] / args.steps
    per_launch_ms = stage_ms[dom] / max(launches, 1)
    n = cls[0].n
    pts = info.valid_points
    if dom == "spread" and args.method == "staged":
        bytes_step = pts * 8 + info.n_valid * n * 8           # point stream in, grid out
        achieved = bytes_step / max(launches, 1) / (per_launch_ms * 1e-3) / 1e9
        roof = {"kernel": "spread_kernel<float>", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None}
    elif dom == "tau":
        bytes_step = pts * 8
        achieved = bytes_step / max(launches, 1) / (per_launch_ms * 1e-3) / 1e9
        roof = {"kernel": "tau_kernel<float>", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None}
    elif dom == "spread":
        ops = algorithmic_ops(cls)
        achieved = ops / max(launches, 1) / (per_launch_ms * 1e-3) / 1e12
        if cls[0].method == 3:
            kname = f"nr::spread_runs_kernel<float, {cls[0].degree}, false>"
        else:
            kname = f"nr::spread_kernel<float, {cls[0].degree}, true, false, false>"
        roof = {"kernel": kname, "bound": "alu", "achieved": achieved,
                "peak": VALU_PEAK_TOPS, "unit": "TOP/s", "frac": achieved / VALU_PEAK_TOPS,
                "traffic": committed_traffic(kname) if len(cls) == 1 else None,
                "traffic_unit": "bytes per launch", "ops_per_point": ops / pts,
                "achieved_basis": "algorithmic VALU lane-operations of the per-sample op model "
                                  "(algorithmic_ops) over the HIP-event launch time; peak = 256 CU x 64 lanes x "
                                  "2.4 GHz, one FP32 or FP64 FMA per lane per cycle"}
        # executed VALU instructions (SQ_INSTS_VALU of the committed profile)
        # x 4 cycles each over the SIMD-cycles of the live launch time
        vi = committed_counter(kname, "valu_instructions_per_launch") if len(cls) == 1 else None
        if vi is not None:
            roof["valu_issue_frac_counters"] = vi * 4 / (1024 * 2.4e9 * per_launch_ms * 1e-3)
            roof["valu_issue_basis"] = ("SQ_INSTS_VALU per launch from the committed rocprofv3 summary x 4 cycles "
                                        "per wave64 instruction / (1024 SIMDs x 2.4 GHz x launch time); about 1 "
                                        "means the VALU pipeline is saturated (it can exceed 1 slightly where "
                                        "transcendental instructions issue beside others)")
    else:
        bytes_step = info.n_valid * n * 8 + info.stat_bins * 8
        achieved = bytes_step / max(launches, 1) / (per_launch_ms * 1e-3) / 1e9
        roof = {"kernel": "epilogue_sum_kernel<float>", "bound": "hbm", "achieved": achieved,
                "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                "traffic": None}
    roof["avg_launch_ms"] = per_launch_ms
    out["roofline"] = roof
    if accuracy is not None:
        out["accuracy"] = accuracy
    # spread + FFT HBM figure of the metric: algorithmic bytes of the spread and
    # FFT/epilogue kernels over their summed time
    sf_bytes = spread_fft_bytes(cls, x32.numel() * x32.element_size(), info.stat_bins, 30)
    out["spread_fft_hbm_bytes"] = sf_bytes
    out["spread_fft_hbm_gbs"] = sf_bytes / ((stage_ms["spread"] + stage_ms["epilogue"]) * 1e-3) / 1e9
    out["spread_fft_hbm_frac"] = out["spread_fft_hbm_gbs"] / HBM_PEAK_GBS

    # the plain FP64 path at the same tolerance
    if not args.no_fp64:
        log("timing fp64")
        p64 = Plan.from_workload(w32, tol=1e-6, precision="fp64", method=args.method, profile=True)
        x64 = p64.strain_tensor(w32.strain, dev)
        s64 = torch.zeros(p64.info.stat_bins, dtype=torch.float64, device=dev)
        u64 = torch.zeros(p64.n_tmpls, dtype=torch.int32, device=dev)
        el64, st64 = time_steps(p64, x64, s64, u64, max(3, args.steps // 2), 1)
        v64 = p64.info.n_valid * max(3, args.steps // 2) / el64
        out["fp64_value"] = v64
        out["speedup_vs_fp64"] = value / v64
        out["fp64_stage_ms_per_step"] = {k: v[0] / max(3, args.steps // 2) for k, v in st64.items()}
        p64.close()

    # the GPU direct non-uniform DFT (no spreading, no FFT) on the same input
    if not args.no_direct:
        log("timing direct-sum baseline")
        pd = Plan.from_workload(w32, tol=1e-6, precision="fp32", method="direct", profile=True)
        sd = torch.zeros(pd.info.stat_bins, dtype=torch.float32, device=dev)
        ud = torch.zeros(pd.n_tmpls, dtype=torch.int32, device=dev)
        nd_steps = max(2, args.steps // 5)
        eld, _ = time_steps(pd, x32, sd, ud, nd_steps, 1)
        sd.zero_()
        ud.zero_()
        pd.semicoherent_sum(x32, None, sd, ud)
        stat.zero_()
        used.zero_()
        plan.semicoherent_sum(x32, None, stat, used)
        torch.cuda.synchronize()
        sa = stat.double().view(-1, 30)
        sb = sd.double().view(-1, 30)
        keep = used > 0
        dst = (torch.linalg.vector_norm(sa - sb, dim=1)[keep] / torch.linalg.vector_norm(sb, dim=1)[keep]).max()
        vd = pd.info.n_valid * nd_steps / eld
        out["direct_baseline"] = {"value": vd, "unit": "spectra/s", "ms_per_step": eld / nd_steps * 1e3,
                                  "nufft_speedup": value / vd, "stat_rel_l2_max_vs_nufft": float(dst),
                                  "kind": "GPU direct non-uniform DFT, FP32, same input and outputs"}
        pd.close()

    # oracle on a bounded seeded sample of instances, on the host cores
    if not args.no_cpu_baseline:
        import oracle
        log("cpu baseline (oracle)")
        rng = np.random.default_rng(123)
        ok_mask = plan.valid_mask().astype(bool)
        cand = np.flatnonzero(ok_mask)
        idx = np.sort(rng.choice(cand, size=min(args.cpu_sample, len(cand)), replace=False))
        t0 = time.perf_counter()
        Xr, off, ok = oracle.spectra(w32, inst_idx=idx)
        t1 = time.perf_counter()
        out["cpu_baseline"] = {"value": len(idx) / (t1 - t0), "unit": "spectra/s",
                               "cores": int(oracle.num_threads()), "kind": "oracle",
                               "sample": f"{len(idx)} seeded valid instances of the {info.n_inst} "
                                         f"(direct long-double sums, {w.seg_len[0]} samples x 30 bins each)",
                               "seconds": t1 - t0}
        sp32, _, _ = plan.execute(x32, want=("spectra",))
        torch.cuda.synchronize()
        X = complex_view(sp32).cpu().numpy().astype(np.complex128)
        boff = plan.bin_offsets()
        errs = []
        for j, i in enumerate(idx):
            g = X[boff[i]:boff[i + 1]]
            r = Xr[off[j]:off[j + 1]]
            errs.append(np.linalg.norm(g - r) / np.linalg.norm(r))
        out["oracle_check"] = {"instances": len(idx), "spectra_rel_l2_max": float(np.max(errs))}
    plan.close()

    # the paper's own beta-bank workload and the ragged batch, timed the same way
    if not args.no_extra:
        for name in ("paper_beta_bank", "ragged_512"):
            # the ragged batch is planned with the autotuner (spreader configuration and
            # FFT radix plan per shape, timed on this GPU at plan creation)
            tuned = name == "ragged_512"
            r = measure_workload(args, dev, name, max(5, args.steps), check=4, tune=tuned)
            out[name] = {k: r[k] for k in ("value", "ms_per_step", "samples_per_s", "spread_ms_per_step",
                                           "spread_valu_frac", "spread_valu_issue_frac_counters",
                                           "oracle_check") if k in r}
            out[name]["workload"] = r["config"]["workload"]
            out[name]["unit"] = "spectra/s"
            out[name]["instances"] = r["config"]["instances"]
            if tuned:
                out[name]["tuned"] = True
                out[name]["plan_seconds_with_tuning"] = r["config"]["plan_seconds"]
                u = measure_workload(args, dev, name, max(5, args.steps), check=0)
                out[name]["untuned_ms_per_step"] = u["ms_per_step"]
        out["mlp_train_step"] = mlp_step_timing(dev)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
