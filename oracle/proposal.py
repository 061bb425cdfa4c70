"""FP64 oracle of the learned proposal's ranking steps -- TEST INFRASTRUCTURE ONLY.

Plain numpy definitions of the steps around the network: the standardised
segment sum, the region features built from it, the largest value of a
group of templates, and the top-k selection.  Only the tests and the
benchmark's CPU leg may use it; the product path never does.

The statistic is the semicoherent sum of Sec. III.C (Eq.
(semicoherent_statistic), unit weights).  For white Gaussian noise of
variance sigma^2, one segment's |X_k|^2 / (L sigma^2) is exponentially
distributed with unit mean (the chi-square with two degrees of freedom of
Sec. III.C, halved), so a sum S over N segments standardises to
    z = (S norm - N) / sqrt(N),   norm = 1 / (L sigma^2),
with mean 0 and variance 1; z = 0 when N = 0.

Readings (the network's inputs and the ranking are not in the paper):
  - region (mc, sb) of a coarse grid of n_mc chirp masses x n_sub sub-bands;
    its feature patch holds z of the 8 chirp masses mc - 3 .. mc + 4
    (clamped to the grid) of sub-band sb at the 8 bins k* - 3 .. k* + 4
    (clamped), k* the lowest bin of the largest summed power of (mc, sb);
    feature 8 i + c is chirp mass i, bin c of the patch;
  - top-k: decreasing score, equal scores in increasing index order, NaN
    last, -0 equal to +0.
"""
from __future__ import annotations

import numpy as np


def zstat(stat, used, K, norm):
    """z [T][K] from summed power stat [T * K] and segment counts used [T]."""
    S = np.asarray(stat, dtype=np.float64).reshape(-1, K)
    N = np.asarray(used, dtype=np.float64).reshape(-1, 1)
    z = np.zeros_like(S)
    pos = N[:, 0] > 0
    z[pos] = (S[pos] * norm - N[pos]) / np.sqrt(N[pos])
    return z


def region_features(stat, used, n_mc, n_sub, K, norm):
    """Features [n_mc * n_sub][64] of every region, template (mc, sb) stored at mc * n_sub + sb."""
    S = np.asarray(stat, dtype=np.float64).reshape(n_mc, n_sub, K)
    z = zstat(stat, used, K, norm).reshape(n_mc, n_sub, K)
    out = np.zeros((n_mc * n_sub, 64))
    for mc in range(n_mc):
        for sb in range(n_sub):
            kstar = int(np.argmax(S[mc, sb]))          # first of the largest
            f = out[mc * n_sub + sb]
            for i in range(8):
                m2 = min(max(mc - 3 + i, 0), n_mc - 1)
                for c in range(8):
                    k = min(max(kstar - 3 + c, 0), K - 1)
                    f[8 * i + c] = z[m2, sb, k]
    return out


def max_z(stat, used, group, K, norm):
    """(zmax [G], arg [G]): the largest z over each run of `group` templates and
    their bins, and its position t_in_group * K + k (first on ties)."""
    z = zstat(stat, used, K, norm).reshape(-1, group * K)
    arg = np.argmax(z, axis=1)
    return z[np.arange(len(z)), arg], arg


def topk(scores, k):
    """Indices [rows][k] of the k largest scores of each row, best first."""
    s = np.atleast_2d(np.asarray(scores, dtype=np.float64))
    s = np.where(s == 0.0, 0.0, s)                        # -0 -> +0
    order = np.argsort(-s, axis=1, kind="stable")         # NaN sorts last
    return order[:, :k]
