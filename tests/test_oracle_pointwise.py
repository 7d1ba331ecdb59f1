"""Pins of the oracle's pointwise physics against facts the paper and the
mathematics fix (not against retyped copies of the same formulas)."""
import math

import numpy as np
import pytest

import oracle as O

ULP = np.finfo(float).eps


def _state(rho, v1, v2, p, gamma):
    return np.array([rho, rho * v1, rho * v2, p / (gamma - 1.0) + 0.5 * rho * (v1 * v1 + v2 * v2)])


def _random_states(n, seed, mach2000=True):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        rho = rng.uniform(0.05, 50.0)
        v1, v2 = rng.uniform(-5, 5, 2)
        p = rng.uniform(0.01, 10.0)
        out.append((rho, v1, v2, p))
    if mach2000:  # cold hypersonic jet-core states and hot post-shock states
        out += [(5.0, 800.0, 0.0, 0.4127), (4.3, 800.0, 3.0, 0.4127), (0.5, 0.0, 0.0, 0.4127),
                (20.0, 650.0, -40.0, 1.7e5), (0.03, 1100.0, 200.0, 0.007)]
    return out


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 3.0])
def test_maxwellian_moments(alpha):
    """eq:maxwellians12-5: sum_k M_k = (1-alpha) u, a(M_1 - M_2) = f(u), a(M_3 - M_4) = g(u)."""
    p = O.Params(alpha=alpha)
    for (rho, v1, v2, pr) in _random_states(40, 1):
        u = _state(rho, v1, v2, pr, p.gamma)
        a = 3.7 * (abs(v1) + abs(v2) + 10.0)
        M = O.maxwellians(p, a, u)
        f, g = O.fluxes(p, u)
        scale = np.abs(M).sum(axis=0) + np.abs(u)
        assert np.all(np.abs(M.sum(axis=0) - (1.0 - alpha) * u) <= 8 * ULP * scale)
        assert np.all(np.abs(a * (M[0] - M[1]) - f) <= 8 * ULP * a * scale)
        assert np.all(np.abs(a * (M[2] - M[3]) - g) <= 8 * ULP * a * scale)


def test_eos_round_trip():
    """eq:eos inverted: p(u(rho, v, p)) = p within the cancellation bound E/(rho e) ulp."""
    p = O.Params()
    for (rho, v1, v2, pr) in _random_states(40, 2):
        u = _state(rho, v1, v2, pr, p.gamma)
        bound = 16 * ULP * u[3] * (p.gamma - 1.0)
        assert abs(O.pressure(p, u) - pr) <= bound + 8 * ULP * pr


def _normal_shock(gamma, rho1, p1, ms):
    """Textbook normal-shock relations in the shock frame: upstream speed ms*c1."""
    c1 = math.sqrt(gamma * p1 / rho1)
    w1 = ms * c1
    rho2 = rho1 * (gamma + 1.0) * ms * ms / ((gamma - 1.0) * ms * ms + 2.0)
    p2 = p1 * (2.0 * gamma * ms * ms - (gamma - 1.0)) / (gamma + 1.0)
    w2 = w1 * rho1 / rho2
    return (rho1, w1, p1), (rho2, w2, p2)


@pytest.mark.parametrize("gamma,ms", [(5.0 / 3.0, 3.0), (1.4, 1.7), (5.0 / 3.0, 2000.0)])
def test_flux_rankine_hugoniot(gamma, ms):
    """eq:fluxF / eq:fluxG: a shock with speed s satisfies f(u_l) - f(u_r) = s (u_l - u_r),
    also with a tangential velocity and in the y direction."""
    p = O.Params(gamma=gamma)
    (r1, w1, p1), (r2, w2, p2) = _normal_shock(gamma, 0.5, 0.4127, ms)
    for s in (0.0, -w1 + 3.0, 17.0):
        for vt in (0.0, 0.3 * w1):
            ua = _state(r1, w1 + s, vt, p1, gamma)
            ub = _state(r2, w2 + s, vt, p2, gamma)
            fa, _ = O.fluxes(p, ua)
            fb, _ = O.fluxes(p, ub)
            scale = np.abs(fa) + np.abs(fb) + abs(s) * (np.abs(ua) + np.abs(ub)) + 1e-300
            assert np.all(np.abs((fa - fb) - s * (ua - ub)) <= 1e-10 * scale.max())
            # same shock travelling in y: swap the momentum components
            va = _state(r1, vt, w1 + s, p1, gamma)
            vb = _state(r2, vt, w2 + s, p2, gamma)
            _, ga = O.fluxes(p, va)
            _, gb = O.fluxes(p, vb)
            assert np.all(np.abs((ga - gb) - s * (va - vb)) <= 1e-10 * scale.max())


@pytest.mark.parametrize("alpha", [0.0, 0.25])
def test_kinetic_speed_is_bouchut_bound(alpha):
    """Sec. 2.1: the kinetic speed must make every dM_k/du monotone (Bouchut).  At the
    oracle's kinetic speed the smallest eigenvalue of the four Jacobians is 0; 2% below
    it one is negative."""
    p = O.Params(alpha=alpha, gamma=1.4)
    g = O.Grid(3, 3, 0.1)
    for (rho, v1, v2, pr) in [(1.0, 0.7, -0.2, 1.0), (2.0, -0.1, 1.5, 0.3), (0.4, 3.0, 2.9, 2.0)]:
        u = _state(rho, v1, v2, pr, p.gamma)
        st = np.zeros((20, 3, 3))
        st[0:4] = u[:, None, None]
        a = O.kinetic_speed(p, g, st)

        def min_eig(aa):
            h = 1e-6 * np.maximum(np.abs(u), 1e-3)
            lam = []
            J = np.zeros((4, 4, 4))
            for c in range(4):
                e = np.zeros(4)
                e[c] = h[c]
                J[:, :, c] = (O.maxwellians(p, aa, u + e) - O.maxwellians(p, aa, u - e)) / (2 * h[c])
            for k in range(4):
                lam.extend(np.linalg.eigvals(J[k]).real)
            return min(lam)

        assert abs(min_eig(a)) < 1e-6
        assert min_eig(0.98 * a) < -1e-3


@pytest.mark.parametrize("alpha", [0.0, 1.0 / 3.0, 0.5])
def test_kinetic_speed_max_over_all_nodes(alpha):
    """a_n uses the fastest node of the whole grid, boundary layers included,
    with the factor 2 / (1 - alpha) of the Bouchut bound."""
    p = O.Params(kappa=1.3, alpha=alpha)
    g = O.Grid(6, 5, 0.01)
    st = np.zeros((20, 5, 6))
    st[0:4] = _state(1.0, 0.1, 0.0, 1.0, p.gamma)[:, None, None]
    st[0:4, 4, 5] = _state(0.2, -9.0, 1.0, 0.5, p.gamma)  # corner copy-layer node
    s_corner, bad = O.wave_speed(p, st[0:4, 4, 5])
    assert not bad
    assert O.kinetic_speed(p, g, st) == pytest.approx(1.3 * 2.0 * s_corner / (1.0 - alpha), rel=1e-15)
    assert s_corner == pytest.approx(9.0 + math.sqrt(p.gamma * 0.5 / 0.2), rel=1e-14)


def test_wave_speed_flags_inadmissible():
    p = O.Params()
    _, bad = O.wave_speed(p, np.array([1.0, 0.0, 0.0, -1.0]))
    assert bad
    _, bad = O.wave_speed(p, np.array([-1.0, 0.0, 0.0, 1.0]))
    assert bad


def test_side_theta_limits():
    """Reading R3: the side limiter returns the largest admissible theta."""
    p = O.Params(pos_eps=0.01)
    L = _state(1.0, 0.0, 0.0, 1.0, p.gamma)
    rhoeL = 1.0 / (p.gamma - 1.0)
    # density-only limiting: D increases rho by 1 per unit theta, bound rho_max' = 1.25
    D = np.array([1.0, 0.0, 0.0, 10.0])
    assert O.side_theta(p, L, 0.5, 1.25, rhoeL, D) == pytest.approx(0.25, rel=1e-15)
    # unconstrained direction -> 1
    assert O.side_theta(p, L, 0.5, 10.0, rhoeL, D) == 1.0
    # internal energy limited: D removes energy only; rho e(theta) = rhoeL - theta*X
    X = 3.0 * rhoeL
    D = np.array([0.0, 0.0, 0.0, -X])
    th = O.side_theta(p, L, 0.5, 10.0, rhoeL, D)
    assert th == pytest.approx((1.0 - p.pos_eps) * rhoeL / X, rel=1e-14)
    # the limited state sits on the floor: rho e = eps rhoeL
    v = L + th * D
    assert v[3] - 0.5 * (v[1] ** 2 + v[2] ** 2) / v[0] == pytest.approx(p.pos_eps * rhoeL, rel=1e-12)
    # kinetic-energy injection (quadratic branch): momentum added at fixed E
    D = np.array([0.0, 2.0, 0.0, 0.0])
    th = O.side_theta(p, L, 0.5, 10.0, rhoeL, D)
    v = L + th * D
    assert v[3] - 0.5 * (v[1] ** 2 + v[2] ** 2) / v[0] == pytest.approx(p.pos_eps * rhoeL, rel=1e-12)
    # energy-limited with the density changing too (the eps * rhoeL * rho(theta)
    # term of the constraint moves with theta): density adds 0.2 per unit theta,
    # momentum 2.0, energy -0.8; the returned theta puts the state on the floor
    # rho e = eps * rhoeL and stays below the (loose) density limit
    D = np.array([0.2, 2.0, 0.0, -0.8])
    th = O.side_theta(p, L, 0.5, 10.0, rhoeL, D)
    assert 0.0 < th < 1.0
    v = L + th * D
    assert v[3] - 0.5 * (v[1] ** 2 + v[2] ** 2) / v[0] == pytest.approx(p.pos_eps * rhoeL, rel=1e-12)
    # a larger eps moves the floor, and theta with it
    p2 = O.Params(pos_eps=0.3)
    th2 = O.side_theta(p2, L, 0.5, 10.0, rhoeL, D)
    v = L + th2 * D
    assert th2 < th
    assert v[3] - 0.5 * (v[1] ** 2 + v[2] ** 2) / v[0] == pytest.approx(0.3 * rhoeL, rel=1e-12)
    # non-positive low-order internal energy -> no antidiffusion
    assert O.side_theta(p, L, 0.5, 10.0, 0.0, D) == 0.0
