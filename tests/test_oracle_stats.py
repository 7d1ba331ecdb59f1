"""Pins of the oracle's ensemble statistics (Sec. 3.2 restriction, Sec. 3.4
observables) against library routines, closed forms and brute force."""
import itertools

import numpy as np
import pytest
from scipy.stats import wasserstein_distance

import oracle as O
from paper_2605_25282_amd import inputs


def test_w1_equals_scipy():
    """eq:w1disc is the 1-D optimal-transport distance (eq:w1cont); for equal-size
    empirical laws it equals scipy's wasserstein_distance."""
    rng = np.random.default_rng(0)
    a = rng.gamma(2.0, 1.0, (37, 5, 4))
    b = rng.normal(2.0, 0.7, (37, 5, 4))
    w = O.w1(a, b)
    for j in range(5):
        for i in range(4):
            assert w[j, i] == pytest.approx(wasserstein_distance(a[:, j, i], b[:, j, i]), rel=1e-12)


@pytest.mark.parametrize("m", [1, 2, 3, 5, 6])
def test_w1_brute_force_optimal_coupling(m):
    """For equal-size empirical laws the optimal coupling is a permutation; the sorted
    formula attains the minimum over all m! permutations (eq:w1cont vs eq:w1disc)."""
    rng = np.random.default_rng(m)
    for _ in range(5):
        a, b = rng.normal(size=m), rng.normal(size=m)
        best = min(np.abs(a - b[list(perm)]).mean() for perm in itertools.permutations(range(m)))
        assert O.w1(a[:, None], b[:, None])[0] == pytest.approx(best, rel=1e-13, abs=1e-15)


def test_w1_invariants():
    """W1 of a shifted copy is the shift; W1 >= |difference of means| (Jensen) and
    W1 <= mean |a_m - b_m| for the same-seed pairing (any coupling bounds the optimum)."""
    rng = np.random.default_rng(3)
    a = rng.uniform(0, 5, (64, 30))
    assert np.allclose(O.w1(a, a + 0.37), 0.37, rtol=1e-13)
    b = a + rng.normal(0, 0.5, a.shape)
    w = O.w1(a, b)
    assert np.all(w >= np.abs(O.ensemble_mean(a) - O.ensemble_mean(b)) - 1e-14)
    assert np.all(w <= np.abs(a - b).mean(axis=0) + 1e-14)


def test_mean_std_match_numpy():
    """Eq:mean and the population standard deviation of eq:std (divide by M)."""
    x = inputs.random_fields(11, (50, 6, 7))
    assert np.allclose(O.ensemble_mean(x), np.mean(x, axis=0), rtol=1e-14)
    assert np.allclose(O.ensemble_std(x), np.std(x, axis=0, ddof=0), rtol=1e-12)


def test_restriction_conserves_integral():
    """Sec. 3.2: the block average is exact and conserves the integral of every field."""
    x = inputs.random_fields(12, (3, 16, 24))
    for r in (1, 2, 4):
        c = O.restrict(x, r)
        assert c.shape == (3, 16 // r, 24 // r)
        assert np.allclose(c.sum(axis=(1, 2)) * r * r, x.sum(axis=(1, 2)), rtol=1e-13)
    assert np.array_equal(O.restrict(x, 1), x)
    with pytest.raises(ValueError):
        O.restrict(x, 5)


def test_dirac_ensemble():
    """eq:empirical with A = 0: all realizations coincide, the standard deviation is 0
    and the one-point W1 between two such ensembles is |difference of means|."""
    p = O.Params(kl_amp=0.0)
    w = inputs.WORKLOADS["jet128"]
    g = O.Grid(w.nx, w.ny, w.dx, w.y_min)
    coefs = inputs.kl_coefficients(1, 0, 3)
    st = np.stack([O.init(p, g, c) for c in coefs])
    rho, speed, pr = O.moments(p, st[:, 0:4])
    assert np.all(O.ensemble_std(rho) == 0.0)
    assert np.array_equal(O.w1(rho, rho + 2.0), np.full(rho.shape[1:], 2.0))


def test_moments_of_known_state():
    """Density, speed and pressure of a state built from primitive values."""
    p = O.Params()
    rho, v1, v2, pr = 2.0, 3.0, -4.0, 7.0
    u = np.array([rho, rho * v1, rho * v2, pr / (p.gamma - 1) + 0.5 * rho * 25.0])[:, None, None]
    r, s, q = O.moments(p, u)
    assert r[0, 0] == 2.0 and s[0, 0] == pytest.approx(5.0, rel=1e-15)
    assert q[0, 0] == pytest.approx(7.0, rel=1e-14)


def test_seeded_generator_published_values():
    """SplitMix64 (Steele, Lea, Flood 2014) seeded with 0 begins 0xE220A8397B1DCDAF,
    0x6E789E6AA1B965F4, 0x06C45D188009454F."""
    z = inputs.stream(0, np.arange(3))
    assert [int(v) for v in z] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_seeded_coefficients_nested_and_uniform():
    """Sec. 3.1: realization m's draws depend on (seed, m) only, so batches and
    prefixes are nested; the coefficients are U(-1, 1)."""
    a = inputs.kl_coefficients(5, 0, 100)
    b = inputs.kl_coefficients(5, 40, 20)
    assert np.array_equal(a[40:60], b)
    big = inputs.kl_coefficients(5, 0, 20000)
    assert big.min() >= -1.0 and big.max() < 1.0
    assert big.mean() == pytest.approx(0.0, abs=0.01)
    assert big.var() == pytest.approx(1.0 / 3.0, rel=0.01)
