"""Pins of the oracle's convergence-study observables (eq:strongError, eq:mean,
eq:std, eq:w1disc), comparison operators (eq:cauchy, eq:ref), rate fit
(eq:ratefit) and the quantile diagnostics (eq:empcdf, eq:widthratio): the
paper's printed Tables 1-7, closed forms, library routines and brute force."""
import os

import numpy as np
import pytest
from scipy.stats import norm

import oracle as O

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "convergence_tables.txt")
OBS = ["W11", "W12", "E_mean", "E_std", "E_strong"]


def _tables():
    rows = []
    for line in open(GOLDEN):
        if line.startswith("#") or not line.strip():
            continue
        t, proto, kind, a, b, *vals = line.split()
        rows.append((float(t), proto, kind, int(a), int(b), [float(v) for v in vals]))
    return rows


def _blocks():
    """(t, protocol) -> (pairs [(coarse Nx, fine Nx, errors)], printed rates)."""
    out = {}
    for t, proto, kind, a, b, vals in _tables():
        pairs, rates = out.setdefault((t, proto), ([], None))
        if kind == "pair":
            pairs.append((a, b, vals))
        else:
            out[(t, proto)] = (pairs, vals)
    return out


def test_golden_tables_complete():
    blocks = _blocks()
    assert len(blocks) == 14  # 7 times x 2 protocols (Tables 1-7)
    for (t, proto), (pairs, rates) in blocks.items():
        assert len(pairs) == 3 and rates is not None and len(rates) == 5


@pytest.mark.parametrize("proto", ["cauchy", "reference"])
def test_comparison_pairs_match_the_tables(proto):
    """eq:cauchy compares successive levels (error at the coarser width), eq:ref each
    level with the finest; the tables list exactly those pairs, coarse first."""
    nx = [500, 1000, 2000, 4000]
    pairs = O.cauchy_pairs(3) if proto == "cauchy" else O.reference_pairs(3)
    got = [(nx[c], nx[f], nx[w]) for c, f, w in pairs]
    for (t, p), (tab, _) in _blocks().items():
        if p == proto:
            assert [(a, b, a) for a, b, _ in tab] == got


def test_rate_fit_reproduces_all_printed_rates():
    """eq:ratefit applied to the printed per-pair errors (4 significant digits)
    reproduces every printed rate of Tables 1-7 (3 decimals): 70 slopes."""
    n = 0
    for (t, proto), (pairs, rates) in _blocks().items():
        dx = [2.5 / a for a, _, _ in pairs]  # mesh width of the coarser member
        for k, obs in enumerate(OBS):
            r, _ = O.rate_fit([v[k] for _, _, v in pairs], dx)
            assert abs(r - rates[k]) <= 1.5e-3, (t, proto, obs, r, rates[k])
            n += 1
    assert n == 70


def test_rate_fit_exact_power_law_and_intercept():
    dx = np.array([0.1, 0.05, 0.025, 0.0125])
    r, c = O.rate_fit(3.7 * dx ** 0.66, dx)
    assert r == pytest.approx(0.66, abs=1e-13) and c == pytest.approx(np.log(3.7), abs=1e-12)
    # a plausible slip (fitting log dx against log E) changes the answer
    r2, _ = O.rate_fit(3.7 * dx ** 0.66 * np.array([1.0, 1.1, 0.95, 1.0]), dx)
    assert abs(r2 - 0.66) > 1e-3


def test_strong_error_properties():
    rng = np.random.default_rng(3)
    M, ny, nx = 9, 6, 7
    f = rng.uniform(0.5, 3.0, (M, ny, nx))
    assert O.strong_error(f, f) == 0.0
    eps = rng.uniform(-0.3, 0.3, M)
    c = f * (1.0 + eps)[:, None, None]
    # a uniformly scaled realization has relative L1 error |eps_m|; averaged over m
    assert O.strong_error(c, f) == pytest.approx(np.abs(eps).mean(), rel=1e-13)
    # normalised by the finer member, not symmetric
    assert O.strong_error(f, c) == pytest.approx(np.mean(np.abs(eps) / (1 + eps)), rel=1e-13)
    # a realization mismatch (pairing different seeds) is not what is measured
    shuffled = f[::-1]
    assert O.strong_error(shuffled, f) > 0.1
    # invariant under a common change of units and under cell permutations
    assert O.strong_error(7.0 * c, 7.0 * f) == pytest.approx(O.strong_error(c, f), rel=1e-13)
    perm = rng.permutation(ny * nx)
    cp, fp = c.reshape(M, -1)[:, perm], f.reshape(M, -1)[:, perm]
    assert O.strong_error(cp, fp) == pytest.approx(O.strong_error(c, f), rel=1e-13)


def test_cell_mean_abs_diff_and_w11():
    rng = np.random.default_rng(4)
    x = rng.normal(size=(5, 8))
    assert O.cell_mean_abs_diff(x + 0.25, x) == pytest.approx(0.25, rel=1e-14)
    assert O.cell_mean_abs_diff(x, -x) == pytest.approx(2 * np.abs(x).mean(), rel=1e-14)
    # W11 of two laws shifted by a constant is that constant (every cell)
    a = rng.gamma(2.0, 1.0, (30, 4, 5))
    assert O.w11(a + 0.5, a) == pytest.approx(0.5, rel=1e-13)
    # W11 >= |difference of the means| cell by cell (Jensen), so also on average
    b = rng.normal(2.0, 0.7, (30, 4, 5))
    assert O.w11(a, b) >= O.cell_mean_abs_diff(O.ensemble_mean(a), O.ensemble_mean(b)) - 1e-15


def test_quantile_small_examples():
    s = np.array([[3.0], [1.0], [2.0], [4.0]])  # M = 4, one cell
    # ceil(alpha M): 5% -> 1, 16% -> 1, 25% -> 1, 26% -> 2, 50% -> 2, 84% -> 4, 100% -> 4
    for pct, want in [(5, 1.0), (16, 1.0), (25, 1.0), (26, 2.0), (50, 2.0), (51, 3.0), (75, 3.0),
                      (76, 4.0), (84, 4.0), (95, 4.0), (100, 4.0)]:
        assert O.empirical_quantile(s, pct)[0] == want, pct
    # ties: hat F jumps by the multiplicity
    t = np.array([[1.0], [2.0], [2.0], [2.0], [5.0]])
    assert O.empirical_quantile(t, 20)[0] == 1.0
    assert O.empirical_quantile(t, 21)[0] == 2.0
    assert O.empirical_quantile(t, 80)[0] == 2.0
    assert O.empirical_quantile(t, 81)[0] == 5.0


@pytest.mark.parametrize("M", [1, 2, 7, 64, 100, 1000])
def test_quantile_is_the_order_statistic(M):
    """eq:empcdf's infimum is the ceil(alpha M)-th order statistic (1-based)."""
    rng = np.random.default_rng(M)
    x = rng.gamma(1.5, 2.0, (M, 3, 4))
    if M > 2:
        x[1] = x[0]  # a tie
    s = np.sort(x, axis=0)
    for pct in (1, 5, 16, 33, 50, 84, 95, 99, 100):
        k = -(-pct * M // 100)
        assert np.array_equal(O.empirical_quantile(x, pct), s[k - 1]), (M, pct)


def test_width_ratio_of_gaussian_laws():
    """Q is the Gaussian constant Q_N = 1.654 for any normal law (eq:widthratio),
    whatever its mean and variance; here from 20000 samples per cell."""
    qn = (norm.ppf(0.95) - norm.ppf(0.05)) / (norm.ppf(0.84) - norm.ppf(0.16))
    assert qn == pytest.approx(1.654, abs=5e-4)
    rng = np.random.default_rng(7)
    z = rng.standard_normal((20000, 2, 3))
    x = z * np.array([0.1, 3.0, 50.0])[None, None, :] + np.array([[-4.0], [9.0]])[None]
    q = O.width_ratio(x)
    assert np.all(np.abs(q - qn) < 0.04)
    # heavier tails raise Q (Student t with 3 degrees of freedom)
    tq = O.width_ratio(rng.standard_t(3, (20000, 1, 1)))[0, 0]
    assert tq > qn + 0.2


@pytest.mark.parametrize("M", [1, 2, 3, 5, 7])
def test_w1_2d_brute_force(M):
    """The assignment optimum equals the minimum over all M! permutations (the
    optimal coupling of two uniform M-point laws is a permutation)."""
    import itertools
    rng = np.random.default_rng(10 + M)
    for _ in range(4):
        p, q = rng.normal(size=(M, 2)), rng.gamma(2.0, 1.0, (M, 2))
        best = min(sum(np.hypot(*(p[i] - q[s[i]])) for i in range(M)) for s in itertools.permutations(range(M)))
        assert O.w1_2d(p, q) == pytest.approx(best / M, rel=1e-13)


def test_w1_2d_special_cases():
    rng = np.random.default_rng(11)
    p = rng.normal(size=(40, 2))
    # a rigid translation by d costs exactly |d| (triangle inequality bound is attained)
    d = np.array([0.3, -1.2])
    assert O.w1_2d(p, p + d) == pytest.approx(np.hypot(*d), rel=1e-13)
    # points on the diagonal: Euclidean distance is sqrt(2)|x - y|, so W is sqrt(2) W1 of the values
    x, y = rng.gamma(2.0, 1.0, 40), rng.normal(3.0, 1.0, 40)
    pd_, qd = np.stack([x, x], 1), np.stack([y, y], 1)
    assert O.w1_2d(pd_, qd) == pytest.approx(np.sqrt(2) * O.w1(x[:, None], y[:, None])[0], rel=1e-12)
    # symmetric and zero on equal laws (any order)
    q = rng.normal(size=(40, 2))
    assert O.w1_2d(p, q) == pytest.approx(O.w1_2d(q, p), rel=1e-13)
    assert O.w1_2d(p, p[rng.permutation(40)]) == 0.0


def test_w12_structure():
    """Subsample indices, pair count and symmetry of eq:w2."""
    assert list(O.subsample_indices(100, 10)) == [5, 15, 25, 35, 45, 55, 65, 75, 85, 95]
    assert list(O.subsample_indices(16, 4)) == [2, 6, 10, 14]
    assert list(O.subsample_indices(7, 7)) == list(range(7))
    rng = np.random.default_rng(12)
    a = rng.gamma(2.0, 1.0, (6, 8, 12))
    b = a + rng.normal(0.0, 0.1, a.shape)
    mean, vals = O.w12(a, b, n_pd=3)
    assert vals.size == 81 and mean == pytest.approx(vals.mean(), rel=1e-14)
    v = vals.reshape(9, 9)
    assert np.allclose(v, v.T, rtol=1e-13, atol=0)  # (k, k') and (k', k) are mirror laws
    # diagonal pairs reduce to sqrt(2) x the one-point W1 of the retained cells
    jy, ix = O.subsample_indices(8, 3), O.subsample_indices(12, 3)
    diag = [np.sqrt(2) * O.w1(a[:, j:j + 1, i], b[:, j:j + 1, i])[0] for j in jy for i in ix]
    assert np.allclose(np.diag(v), diag, rtol=1e-12, atol=0)
    assert O.w12(a, a, n_pd=3)[0] == 0.0
