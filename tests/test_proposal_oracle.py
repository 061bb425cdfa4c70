"""Pins of the proposal oracle (oracle/proposal.py) against facts that do not
come from the oracle itself: the chi-square noise law of the power (Sec.
III.C), inputs built backwards from chosen statistics, brute-force orderings
and hand-placed cases for every index and clamp of the feature patch."""
import numpy as np
import pytest

from oracle import proposal as op


def _stat_from_z(z, used, norm):
    """Summed power that standardises to z: S = (N + z sqrt(N)) / norm."""
    N = np.asarray(used, np.float64)[:, None]
    return ((N + z * np.sqrt(N)) / norm).ravel()


def test_noise_sums_standardise_to_unit_normal():
    """|X|^2 of N(0,1) noise over L samples is (L/2) chi^2_2 (Sec. III.C): sums over
    N segments, standardised with norm = 1/L, have mean 0 and variance 1."""
    rng = np.random.default_rng(3)
    L, N, T, K = 7680, 40, 2000, 30
    S = (0.5 * L) * rng.chisquare(2.0, size=(T, N, K)).sum(axis=1)
    z = op.zstat(S.ravel(), np.full(T, N), K, 1.0 / L)
    assert abs(z.mean()) < 0.01 and abs(z.var() - 1.0) < 0.02
    # the sum of N unit exponentials is Gamma(N): its skewness 2/sqrt(N) survives
    skew = np.mean(z ** 3)
    assert abs(skew - 2 / np.sqrt(N)) < 0.03


def test_zstat_inverts_and_zero_count():
    rng = np.random.default_rng(4)
    used = np.array([5, 0, 120, 1])
    z = rng.standard_normal((4, 7))
    got = op.zstat(_stat_from_z(z, used, 0.25), used, 7, 0.25)
    z[1] = 0.0                                     # N = 0 gives z = 0
    assert np.allclose(got, z, rtol=0, atol=1e-12)


def test_region_features_patch_positions_and_clamps():
    """A grid whose z encodes (chirp mass, sub-band, bin) so that every feature
    names the template and bin it came from; the loudest bin of each template
    is placed by hand, including at both edges of the band."""
    n_mc, n_sub, K, norm = 6, 3, 12, 0.5
    used = np.full(n_mc * n_sub, 9)
    code = lambda m, b, k: 1000.0 * m + 100.0 * b + k      # distinct for every cell
    z = np.array([[code(m, b, k) for k in range(K)] for m in range(n_mc) for b in range(n_sub)])
    # loudest bin of template (m, b): make z larger there than elsewhere in its row
    loud = {(m, b): [0, 5, 11][(m + b) % 3] for m in range(n_mc) for b in range(n_sub)}
    for (m, b), k in loud.items():
        z[m * n_sub + b, k] += 50.0
    S = _stat_from_z(z, used, norm)
    f = op.region_features(S, used, n_mc, n_sub, K, norm)
    for m in range(n_mc):
        for b in range(n_sub):
            ks = loud[(m, b)]
            for i in range(8):
                m2 = min(max(m - 3 + i, 0), n_mc - 1)
                for c in range(8):
                    k = min(max(ks - 3 + c, 0), K - 1)
                    want = code(m2, b, k) + (50.0 if loud[(m2, b)] == k else 0.0)
                    assert f[m * n_sub + b, 8 * i + c] == pytest.approx(want, abs=1e-8)


def test_region_features_first_of_equal_maxima():
    n_mc, n_sub, K = 1, 1, 10
    S = np.ones(K)
    S[[2, 7]] = 4.0
    f = op.region_features(S, np.array([1]), n_mc, n_sub, K, 1.0)
    # k* = 2: the patch covers bins clamp(-1..6) -> 0, 0, 1, 2, 3, 4, 5, 6 with z = S - 1
    want = np.array([0, 0, 1, 2, 3, 4, 5, 6])
    assert np.array_equal(f[0, :8], S[want] - 1.0)


def test_max_z_brute_force_and_ties():
    rng = np.random.default_rng(5)
    G, group, K = 7, 3, 5
    used = rng.integers(0, 4, size=G * group)
    used[[4, 5]] = 2
    z = rng.standard_normal((G * group, K))
    z[used == 0] = 0.0
    z[4, 2] = z[5, 1] = 9.0                        # a tie inside group 1: first position wins
    S = _stat_from_z(z, np.maximum(used, 0), 1.0)
    zm, arg = op.max_z(S, used, group, K, 1.0)
    for g in range(G):
        best, where = -np.inf, -1
        for t in range(group):
            for k in range(K):
                v = z[g * group + t, k]
                if v > best + 1e-9:
                    best, where = v, t * K + k
        assert zm[g] == pytest.approx(best, abs=1e-9) and arg[g] == where
    assert arg[1] == (4 - 3) * K + 2


def test_topk_orders_permutations_ties_nan_and_signed_zero():
    rng = np.random.default_rng(6)
    perm = rng.permutation(50).astype(np.float64)
    assert np.array_equal(op.topk(perm, 50)[0], np.argsort(perm)[::-1])
    s = np.array([1.0, 3.0, np.nan, 3.0, -0.0, 0.0, -2.0, 3.0])
    assert op.topk(s, 8)[0].tolist() == [1, 3, 7, 0, 4, 5, 6, 2]
    rows = rng.standard_normal((4, 9))
    top = op.topk(rows, 3)
    for r in range(4):
        assert set(top[r]) == set(np.argsort(rows[r])[-3:])
