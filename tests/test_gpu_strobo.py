"""Parity of the stroboscopic baseline (through the C ABI) with its oracle:
the nearest-neighbour fold is bit-exact against the same fold computed on
the host from the oracle's nearest indices (float32 adds in the same order),
and the baseline's spectrum matches the oracle's direct sum to 2e-6."""
import sys

import numpy as np
import pytest

import synth
from oracle import strobo as ost

pytestmark = pytest.mark.gpu


def say(m):
    print(m, flush=True)
    sys.stdout.flush()


@pytest.mark.parametrize("mc,cplx", [(0.0, False), (1e-1, True), (1e-1, False), (3e-2, True)])
def test_fold_and_spectrum_match_oracle(gpu, mc, cplx):
    import torch
    from paper_2609_12476_amd import strobo
    say(f"strobo mc={mc} complex={cplx}")
    fs, T, O, f0 = 128.0, 16.0, 8, 20.0
    fs_o = fs * O
    n = int(round(T * fs_o))
    rng = np.random.default_rng(9)
    t = np.arange(n) / fs_o
    if cplx:
        x = 0.5 * np.exp(1j * synth.chirp_phase(t, f0, max(mc, 1e-30), 0.0, 0.3)) + \
            0.1 * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
        x = x.astype(np.complex64)
    else:
        x = (np.cos(synth.chirp_phase(t, f0, max(mc, 1e-30), 0.0, 0.3)) + 0.1 * rng.standard_normal(n))
        x = x.astype(np.float32)
    xd = torch.from_numpy(x).to(gpu)
    N = int(round(T * fs_o))
    M = strobo.nr_strobo_points(fs_o, n, mc, f0)
    tau, tt = ost.tau_points(mc, f0, fs_o, n)
    assert M == len(tau)
    # two copies of the segment exercise the batch: both folds must be the same
    fold = strobo.nr_strobo_fold(torch.cat([xd, xd]), n, fs_o, mc, f0, N, n_seg=2)
    torch.cuda.synchronize()
    assert torch.equal(fold[0], fold[1])
    fold = fold[0]
    # the same fold on the host: nearest indices of the oracle, float32 adds in m order
    idx = ost.nearest(tt, fs_o, n)
    ref = np.zeros(N, np.complex64)
    for m in range(M):
        if idx[m] >= 0:
            ref[m % N] = np.complex64(ref[m % N] + np.complex64(x[idx[m]]))
    got = fold.cpu().numpy()
    assert np.array_equal(got, ref), int(np.sum(got != ref))
    f_lo, K = 18.0, 64
    S = strobo.spectrum(xd, fs_o, O, mc, f0, f_lo, 1.0 / T, K)[0].cpu().numpy().astype(np.complex128)
    Sr = ost.spectrum(x.astype(np.complex128), fs_o, O, mc, f0, f_lo, 1.0 / T, K)
    e = np.linalg.norm(S - Sr) / np.linalg.norm(Sr)
    say(f"  spectrum rel l2 {e:.2e}")
    assert e <= 2e-6


def test_comparison_shape_sampled(gpu):
    """The comparison's 256 s shape at O = 8 over 32 batched segments: every
    segment's fold equals the first's (same input), and 64 bins around 20 Hz
    match the oracle's direct sum."""
    import torch
    from paper_2609_12476_amd import strobo
    say("strobo 256 s, O = 8, 32 segments")
    f0, mc, fs, O, T = 20.0, 1e-2, 512.0, 8, 256.0
    fs_o = fs * O
    n = int(T * fs_o)
    x = (0.5 * np.exp(1j * synth.chirp_phase(np.arange(n) / fs_o, f0, mc, 0.0, 0.3))).astype(np.complex64)
    xd = torch.from_numpy(x).to(gpu).repeat(32)
    df = 1.0 / T
    lo = 20.0 - 32 * df
    S = strobo.spectrum(xd, fs_o, O, mc, f0, lo, df, 64, n_seg=32)
    torch.cuda.synchronize()
    S = S.cpu().numpy().astype(np.complex128)
    assert np.allclose(S[0], S[-1], rtol=1e-6, atol=1e-6 * np.abs(S[0]).max())
    ref = ost.spectrum(x.astype(np.complex128), fs_o, O, mc, f0, lo, df, 64)
    e = np.linalg.norm(S[0] - ref) / np.linalg.norm(ref)
    say(f"  rel l2 {e:.2e}")
    assert e <= 2e-6
