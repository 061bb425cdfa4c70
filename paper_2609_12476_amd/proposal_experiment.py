"""Train the learned proposal and judge it against exhaustive refinement.

    python -m paper_2609_12476_amd.proposal_experiment --out results.json [--scale 0.1]

Steps (all on one GPU):
  1. training set: one draw per coarse region per batch, half with an injection
     placed in that region (SNR uniform 4-20), half noise only; features from
     the 8-cell window around the region (WindowPlan).
  2. train the network with minibatch Adam on the GPU kernels.
  3. detection threshold: the (1 - 1e-2) quantile over noise-only draws of the
     exhaustive search's maximum z over every fine template.
  4. held-out injections: blind coarse grid -> features -> logits; regions are
     ranked by the network and, as the non-learned baseline, by their largest
     coarse z.  A search detects an injection if some fine template of a
     region it refines within one cell of the true region (same sub-band)
     reaches the threshold; the exhaustive search refines every region.
Reports the missed-injection rates at several k, the extra misses against
exhaustive search, and the refined-grid cost fraction k / regions.
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np


def log(m):
    print(m, file=sys.stderr, flush=True)


def run(scale=1.0, n_mc=256, per_cell=8, ks=(32, 128, 512), epochs=30, seed=1234, dev="cuda:0"):
    import torch

    from . import proposal as pp
    from .mlp import Mlp

    torch.manual_seed(seed)
    gen = torch.Generator(device=dev).manual_seed(seed)
    grid = pp.Grid(n_mc)
    n_regions = n_mc * pp.N_SUB
    n_train = int(round(1e5 * scale))            # per class (injection / noise)
    n_judge = int(round(2e4 * scale))
    n_thr = max(100, int(round(1000 * scale)))
    out = {"n_mc_coarse": n_mc, "fine_per_cell": per_cell, "regions": n_regions,
           "train_per_class": n_train, "held_out_injections": n_judge, "threshold_noise_draws": n_thr}
    t_start = time.time()

    # ---------------------------------------------------------------- 1. data
    # one slot per coarse region; a batch is all-injection or all-noise
    all_regions = np.arange(n_regions)
    m_all, b_all = all_regions // pp.N_SUB, all_regions % pp.N_SUB
    wp = pp.WindowPlan(grid, (m_all, b_all))
    rng = np.random.default_rng(seed)
    X, Y = [], []
    done = [0, 0]
    while done[0] < n_train or done[1] < n_train:
        label = 1 if done[1] <= done[0] else 0
        take = min(n_regions, n_train - done[label])
        inj = pp.draw_injections(gen, (m_all, b_all), grid) if label else None
        x = pp.make_strain(gen, n_regions, inj)
        f, _, _ = wp.features(x)
        keep = torch.as_tensor(np.sort(rng.choice(n_regions, size=take, replace=False)), device=f.device)
        X.append(f[keep].clone())
        Y.append(torch.full((take,), float(label), device=f.device))
        done[label] += take
        del x, f
        log(f"training data: {done[1]} injections, {done[0]} noise")
    X = torch.cat(X)
    Y = torch.cat(Y)
    wp.plan.close()
    torch.cuda.synchronize()
    out["data_seconds"] = time.time() - t_start

    # --------------------------------------------------------------- 2. train
    import synth
    net = Mlp(max_batch=1024, params=synth.mlp_init_params(seed))
    t0 = time.time()
    hist = pp.train(net, X, Y, epochs=epochs, batch=1024, lr=1e-3, seed=seed, log=log)
    torch.cuda.synchronize()
    out["train_seconds"] = time.time() - t0
    out["loss_history"] = hist
    with torch.no_grad():
        z = net.forward(X)
        out["train_accuracy"] = float(((z > 0).float() == Y).float().mean())
    del X, Y

    # ----------------------------------------------------------- 3. threshold
    fine_mc = np.concatenate([grid.fine(m, per_cell) for m in range(n_mc)])
    D_thr = 2
    all_mc = np.tile(np.repeat(fine_mc, pp.N_SUB), D_thr)
    all_sb = np.tile(np.tile(np.arange(pp.N_SUB), len(fine_mc)), D_thr)
    fp_all = pp.FinePlan(all_mc, all_sb, D_thr)
    maxes = []
    t0 = time.time()
    for i in range(0, n_thr, D_thr):
        x = pp.make_strain(gen, D_thr)
        mz = fp_all.max_z(x)
        maxes.append(mz.amax(dim=1).cpu())
    fp_all.plan.close()
    maxes = torch.cat(maxes).numpy()[:n_thr]
    thr = float(np.quantile(maxes, 1 - 1e-2))
    out["threshold_z"] = thr
    out["threshold_seconds"] = time.time() - t0
    log(f"threshold z = {thr:.3f} from {len(maxes)} noise draws")

    # ------------------------------------------------------------ 4. judging
    D_j = 16
    cp = pp.CoarsePlan(grid, D_j)
    det_exh = []
    det_learn = {k: [] for k in ks}
    det_base = {k: [] for k in ks}
    t0 = time.time()
    for i0 in range(0, n_judge, D_j):
        reg = rng.choice(all_regions, size=D_j, replace=True)
        m, b = reg // pp.N_SUB, reg % pp.N_SUB
        inj = pp.draw_injections(gen, (m, b), grid)
        x = pp.make_strain(gen, D_j, inj)
        feats, stat, used = cp.run(x)
        logits = net.forward(feats.view(-1, 64)).view(D_j, n_regions)
        zc = pp.zstat(stat, used).amax(dim=2)                   # [D][regions]
        # fine templates of the true region and its neighbours (same sub-band)
        nb_cells = np.clip(m[:, None] + np.array([-1, 0, 1])[None, :], 0, n_mc - 1)   # [D][3]
        mcs = np.stack([np.concatenate([grid.fine(c, per_cell) for c in row]) for row in nb_cells])
        subs = np.repeat(b[:, None], 3 * per_cell, axis=1)
        fp = pp.FinePlan(mcs.ravel(), subs.ravel(), D_j)
        fz = fp.max_z(x).view(D_j, 3, per_cell).amax(dim=2).cpu().numpy()  # [D][3] per neighbour
        fp.plan.close()
        nb_region = nb_cells * pp.N_SUB + b[:, None]
        lg = logits.cpu().numpy()
        zcn = zc.cpu().numpy()
        for d in range(D_j):
            hit = fz[d] >= thr
            det_exh.append(bool(hit.any()))
            for k in ks:
                # ties: lower region index first (stable sort on the negated score)
                sel_l = set(np.argsort(-lg[d], kind="stable")[:k].tolist())
                sel_b = set(np.argsort(-zcn[d], kind="stable")[:k].tolist())
                det_learn[k].append(bool(any(hit[q] and nb_region[d, q] in sel_l for q in range(3))))
                det_base[k].append(bool(any(hit[q] and nb_region[d, q] in sel_b for q in range(3))))
        del x
        if (i0 // D_j) % 50 == 0:
            log(f"judged {i0 + D_j}/{n_judge}")
    cp.plan.close()
    out["judge_seconds"] = time.time() - t0
    n = len(det_exh)
    miss_exh = 1 - np.mean(det_exh)
    out["missed_exhaustive"] = miss_exh
    out["by_k"] = []
    for k in ks:
        ml = 1 - np.mean(det_learn[k])
        mb = 1 - np.mean(det_base[k])
        out["by_k"].append({"k": k, "refined_fraction": k / n_regions,
                            "missed_learned": ml, "missed_baseline": mb,
                            "extra_missed_learned": ml - miss_exh,
                            "extra_missed_baseline": mb - miss_exh})
    out["held_out_judged"] = n
    out["total_seconds"] = time.time() - t_start
    net.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default=None)
    ap.add_argument("--scale", type=float, default=1.0)
    ap.add_argument("--epochs", type=int, default=30)
    args = ap.parse_args()
    res = run(scale=args.scale, epochs=args.epochs)
    s = json.dumps(res)
    if args.out:
        with open(args.out, "w") as f:
            f.write(s + "\n")
    print(s)


if __name__ == "__main__":
    main()
