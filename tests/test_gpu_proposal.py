"""The learned proposal's ranking and refinement steps on the GPU, through the
C ABI, against the oracle.

- nr_prop_topk and nr_prop_max_z on the same float inputs as the oracle:
  selections bit-exact, maxima within one float rounding.
- End to end on a small search (8 segments x 4 sub-bands x 16 coarse chirp
  masses, one injection): coarse segment sums (<= 1e-4 per template, counts
  exact), region features, network logits, top-k of the logits and of the
  coarse z, and the refined regions' best fine z, each against the oracle
  chain built from the oracle's own sums (oracle.semicoherent,
  oracle.proposal, oracle.mlp).  Where floating point decides an integer (the
  loudest bin of a feature patch, the order at the k-th score) the GPU's
  choice must be one the oracle's values allow within the tolerance.
"""
import sys

import numpy as np
import pytest

import oracle
import synth
from oracle import mlp as om
from oracle import proposal as op
from synth import proposal as sp

pytestmark = pytest.mark.gpu


def say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


# ----------------------------------------------------------- kernels alone --

@pytest.mark.parametrize("n,k", [(1, 1), (37, 5), (1280, 32), (5120, 128), (5120, 5120), (16384, 512)])
def test_topk_bit_exact(gpu, n, k):
    import torch
    from paper_2609_12476_amd import proposal as pp
    say(f"topk n={n} k={k}")
    rng = np.random.default_rng(n + k)
    rows = 5
    s = rng.standard_normal((rows, n)).astype(np.float32)
    s[0, : n // 2] = np.round(s[0, : n // 2])            # many ties
    if n > 3:
        s[1, 1], s[1, 2], s[1, 3] = np.nan, -0.0, 0.0       # NaN last, signed zeros equal
    s[2] = 1.0                                            # all equal: ascending items
    got = pp.nr_prop_topk(torch.from_numpy(s).to(gpu), rows, n, k).cpu().numpy()
    want = op.topk(s.astype(np.float64), k)
    assert np.array_equal(got, want)


@pytest.mark.parametrize("group,K", [(1, 30), (8, 30), (3, 600), (64, 7)])
def test_max_z_matches_oracle(gpu, group, K):
    import torch
    from paper_2609_12476_amd import proposal as pp
    say(f"max_z group={group} K={K}")
    rng = np.random.default_rng(group * 1000 + K)
    G = 37
    T = G * group
    used = rng.integers(0, 121, size=T).astype(np.int32)
    used[: group] = 0                                     # a group with no segments: z = 0
    used[5 * group] = 50
    L = 7680
    stat = ((0.5 * L) * rng.chisquare(2.0, size=(T, K)) * np.maximum(used, 1)[:, None]).astype(np.float32)
    stat[5 * group, 3 % K] = stat[5 * group, 1 % K] = 1e7  # ties inside one group
    z, a = pp.nr_prop_max_z(torch.from_numpy(stat.ravel()).to(gpu), torch.from_numpy(used).to(gpu), G, group, K,
                            1.0 / L, arg=torch.empty(G, dtype=torch.int32, device=gpu))
    zr, ar = op.max_z(stat.astype(np.float64).ravel(), used, group, K, 1.0 / L)
    assert np.array_equal(a.cpu().numpy(), ar)
    assert np.allclose(z.cpu().numpy(), zr.astype(np.float32), rtol=2 ** -23, atol=0)


# ------------------------------------------------------------ end to end --

LAY = sp.Layout(n_seg=8, t_coh=30.0, fs=256.0, n_sub=4, band_lo=40.0)
GRID = sp.Grid(16)
PER_CELL, TOP_K = 4, 8
TRUE_REGION = (9, 2)


def _tied_ok(gpu_sel, ora_sel, ora_score, tol):
    """Every region the GPU selects but the oracle does not (and vice versa) must
    score within tol (per region) of the oracle's k-th score."""
    kth = np.sort(ora_score)[::-1][len(ora_sel) - 1]
    tol = np.broadcast_to(np.asarray(tol, np.float64), ora_score.shape)
    diff = set(int(r) for r in gpu_sel) ^ set(int(r) for r in ora_sel)
    return all(abs(ora_score[r] - kth) <= tol[r] for r in diff), diff


def test_proposal_pipeline_end_to_end(gpu):
    import torch
    from paper_2609_12476_amd import proposal as pp
    from paper_2609_12476_amd.mlp import Mlp
    say("proposal pipeline end to end")
    lay, grid = LAY, GRID
    R, K = grid.n_mc * lay.n_sub, lay.K
    x, inj = sp.draw_numpy(lay, grid, TRUE_REGION, seed=11, snr=25.0)
    x32 = x.astype(np.float32).astype(np.float64)         # the values both sides see
    xd = torch.from_numpy(x32).to(device=gpu, dtype=torch.float32).view(1, -1)

    # --- coarse sums -------------------------------------------------------
    cmc = np.repeat(grid.centres(), lay.n_sub)
    csb = np.tile(np.arange(lay.n_sub), grid.n_mc)
    so, soff, uo = oracle.semicoherent(sp.workload(lay, x32, cmc, csb))
    cp = pp.CoarsePlan(lay, grid, 1)
    feats, stat, used = cp.run(xd)
    zc = cp.max_z(stat, used)
    torch.cuda.synchronize()
    S = stat.cpu().numpy().astype(np.float64).reshape(R, K)
    U = used.cpu().numpy()
    assert np.array_equal(U, uo)
    So = so.reshape(R, K)
    for t in range(R):
        if uo[t]:
            e = np.linalg.norm(S[t] - So[t]) / np.linalg.norm(So[t])
            assert e <= 1e-4, (t, e)

    # --- features, where the loudest bin is not a near tie -----------------
    fo = op.region_features(so, uo, grid.n_mc, lay.n_sub, K, lay.norm)
    fg = feats.cpu().numpy().reshape(R, 64).astype(np.float64)
    srt = np.sort(So, axis=1)
    clear = (srt[:, -1] - srt[:, -2]) > 1e-3 * srt[:, -1]
    ztol = 1e-4 * (1.0 + np.abs(fo)) + 1e-4 * np.sqrt(np.max(uo))
    assert clear.sum() >= R // 2
    assert np.all(np.abs(fg - fo)[clear] <= ztol[clear])
    say(f"  features: {clear.sum()} of {R} regions with a clear loudest bin match")

    # --- network logits -----------------------------------------------------
    params = synth.mlp_init_params(3)
    net = Mlp(max_batch=64, params=params)
    top_l, logits = pp.rank(net, feats, TOP_K)
    lo_g = logits.cpu().numpy().ravel().astype(np.float64)
    lo_o, _ = om.forward(om.weights_as_used(params), fo)
    assert np.all(np.abs(lo_g - lo_o)[clear] <= 1e-3 * (1.0 + np.abs(lo_o[clear])))
    # a region without a clear loudest bin may take either bin's patch, so its
    # logit may differ: it may enter or leave the selection
    ltol = 1e-3 * (1.0 + np.abs(lo_o)) + np.where(clear, 0.0, np.inf)

    # --- top-k of the logits and of the coarse z ----------------------------
    sel_g = top_l.cpu().numpy()[0]
    sel_o = op.topk(lo_o, TOP_K)[0]
    ok, diff_l = _tied_ok(sel_g, sel_o, lo_o, ltol)
    assert ok, diff_l
    zcg = zc.cpu().numpy().ravel().astype(np.float64)
    zco, _ = op.max_z(so, uo, 1, K, lay.norm)
    assert np.allclose(zcg, zco, rtol=1e-4, atol=1e-4 * np.sqrt(lay.n_seg))
    selb_g = pp.rank_max_z(zc, TOP_K).cpu().numpy()[0]
    selb_o = op.topk(zco, TOP_K)[0]
    ok, diff = _tied_ok(selb_g, selb_o, zco, 1e-4 * (1 + np.abs(zco).max()))
    assert ok, diff
    true_r = TRUE_REGION[0] * lay.n_sub + TRUE_REGION[1]
    assert true_r in set(selb_o) and true_r in set(selb_g)     # a loud injection ranks high

    # --- refinement of the selected regions ---------------------------------
    fz_g = pp.refine(lay, grid, xd, top_l, PER_CELL).cpu().numpy()[0].astype(np.float64)
    m_o, b_o = sel_o // lay.n_sub, sel_o % lay.n_sub
    fmc = grid.fine_of_regions(m_o, PER_CELL).ravel()
    fsb = np.repeat(b_o, PER_CELL)
    sf, _, uf = oracle.semicoherent(sp.workload(lay, x32, fmc, fsb))
    fz_o, _ = op.max_z(sf, uf, PER_CELL, K, lay.norm)
    common = [r for r in sel_g if r in set(sel_o)]
    assert len(common) >= TOP_K - len(diff_l)
    for r in common:
        a = fz_g[list(sel_g).index(r)]
        b = fz_o[list(sel_o).index(r)]
        assert abs(a - b) <= 1e-4 * (1.0 + abs(b)) + 1e-4 * np.sqrt(lay.n_seg), (r, a, b)
    say(f"  refined {len(common)} common regions; best fine z {fz_g.max():.2f}")
    net.close()
    cp.close()
