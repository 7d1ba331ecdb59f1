"""Pins of the stochastic inlet (eq:rho_inlet_def, eq:karhunenExp) against the
numbers the paper prints (Sec. 2.3, Sec. 4.3, Figure 1)."""
import math
import os

import numpy as np
import pytest

import oracle as O
from paper_2605_25282_amd import inputs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "fig1_inlet_envelope.txt")


def _rho_samples(p, ybar, coefs):
    return np.array([[O.inlet_density(p, yb * p.r_jet, c) for yb in ybar] for c in coefs])


def test_axis_std_matches_paper():
    """Sec. 4.3: on the axis the inlet perturbation has standard deviation
    A rho_jet (sum_k k^-4 / 3)^(1/2) ~ 0.30.  Sampled with M = 40000 realizations."""
    p = O.Params()
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, 40000)
    rho0 = np.array([O.inlet_density(p, 0.0, c) for c in coefs])
    closed = p.kl_amp * p.rho_jet * math.sqrt(sum(k ** -4.0 for k in range(1, 11)) / 3.0)
    assert closed == pytest.approx(0.30, abs=0.005)  # the value the paper prints
    assert rho0.std() == pytest.approx(closed, rel=0.015)
    assert rho0.mean() == pytest.approx(p.rho_jet, abs=4 * closed / math.sqrt(40000))


def test_fig1_envelope():
    """Figure 1: the +-1 sigma band and mean of M = 1000 paper samples, against the
    oracle's inlet density sampled at the same normalised coordinates.  Tolerance:
    sampling noise of the paper's M = 1000 band (~sigma/sqrt(2M) <= 0.007) plus the
    printed 3 decimals; the window W(ybar) = cos^2(pi ybar/2) and the reading of the
    mode argument as pi*k*ybar are what this pins (reading R4, R5)."""
    data = np.loadtxt(GOLDEN)
    ybar, upper, lower, mean = data.T
    p = O.Params()
    coefs = inputs.kl_coefficients(inputs.DEFAULT_SEED, 0, 8000)
    rho = _rho_samples(p, ybar, coefs)
    sig_paper = 0.5 * (upper - lower)
    assert np.abs(rho.std(axis=0) - sig_paper).max() < 0.025
    assert np.abs(rho.mean(axis=0) - mean).max() < 0.02
    # the band collapses onto 5.000 at the jet edge
    assert rho.std(axis=0)[0] < 1e-12 and rho.std(axis=0)[-1] < 1e-12


def test_extreme_mach_numbers():
    """Sec. 2.3: with all coefficients at their bounds the axis density is
    rho_jet (1 +- A sum k^-2) and the internal Mach number, which scales as sqrt(rho),
    varies by +7.5% / -8.1%; at one standard deviation by about +-3%."""
    p = O.Params()
    hi = np.zeros(20)
    hi[0::2] = 1.0          # Y_k = 1, Z_k irrelevant on the axis (sin 0 = 0)
    r_hi = O.inlet_density(p, 0.0, hi)
    r_lo = O.inlet_density(p, 0.0, -hi)
    assert round(100 * (math.sqrt(r_hi / p.rho_jet) - 1), 1) == 7.5
    assert round(100 * (math.sqrt(r_lo / p.rho_jet) - 1), 1) == -8.1
    sigma = p.kl_amp * math.sqrt(sum(k ** -4.0 for k in range(1, 11)) / 3.0)
    assert round(100 * 0.5 * sigma) == 3


def test_inlet_state_structure():
    """Sec. 2.2: step velocity profile, ambient density outside |y| <= r_jet, pressure
    p_amb everywhere (E from eq:eos)."""
    p = O.Params()
    c = inputs.kl_coefficients(7, 0, 1)[0]
    for y in (-0.2, -0.0501, -0.05, -0.03, 0.0, 0.049, 0.05, 0.11):
        u = O.inlet_state(p, y, c)
        inside = abs(y) <= p.r_jet
        assert u[1] == pytest.approx(u[0] * (p.v_jet if inside else 0.0), rel=1e-15)
        assert u[2] == 0.0
        if not inside:
            assert u[0] == p.rho_amb
        assert O.pressure(p, u) == pytest.approx(p.p_amb, rel=1e-9 if inside else 1e-15)
