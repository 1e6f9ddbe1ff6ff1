"""Pins of the oracle's cross-section post-processing (Section III, Eqs. 19-20, rates).

  microscopically reversible input: Eq. 19 ratio 1, Eq. 20 returns g sigma     -> Eq. 19/20 forms
  sigma~ symmetric, linear in sigma                                             -> Eq. 20
  constant cross section (with the threshold ramp and the constant tail):
    closed form through the regularised incomplete gamma function (scipy)      -> Maxwell-Boltzmann
                                                                                  weight, prefactor
  elastic limit, constant sigma everywhere: k = sigma * mean speed / g          -> textbook
  cross section linear in U (the natural spline is exact): closed form        -> spline segments
  detailed balance g' k' exp(-E'/kT) = g'' k'' exp(-E''/kT)                     -> exp(-dE/2kT)
"""
import math

import numpy as np
from scipy import special

from oracle import postproc as PP


def test_eq19_eq20_on_reversible_input():
    rng = np.random.default_rng(0)
    L, nE = 5, 3
    g = rng.integers(1, 20, L).astype(float)
    base = rng.random((nE, L, L))
    W = base + np.swapaxes(base, 1, 2)                  # symmetric g_i sigma_{i->f}
    sigma = W / g[None, :, None]
    r = PP.reversibility_ratio(sigma, g)
    assert np.max(np.abs(r - 1.0)) < 1e-14
    sym = PP.symmetrize(sigma, g)
    assert np.max(np.abs(sym - W)) < 1e-14


def test_eq20_symmetric_and_linear():
    rng = np.random.default_rng(1)
    L, nE = 6, 4
    g = rng.integers(1, 10, L).astype(float)
    a, b = rng.random((nE, L, L)), rng.random((nE, L, L))
    sa, sb = PP.symmetrize(a, g), PP.symmetrize(b, g)
    assert np.array_equal(sa, np.swapaxes(sa, 1, 2))
    assert np.max(np.abs(PP.symmetrize(2 * a - 3 * b, g) - (2 * sa - 3 * sb))) < 1e-14
    r = PP.reversibility_ratio(a, g)
    assert np.max(np.abs(r * np.swapaxes(r, 1, 2) - 1.0)) < 1e-14


def lower_gamma(n, x):
    """int_0^x t^(n-1) e^-t dt."""
    return special.gamma(n) * special.gammainc(n, x)


def test_constant_cross_section_closed_form():
    mu, g_i = 1500.0, 3.0
    U = np.array([0.002, 0.004, 0.008, 0.016])
    c = 7.5
    for dE in (0.0, 0.0015, -0.0015):
        for beta in (0.0005, 0.002, 0.01):
            k = PP.rate_coefficient(U, np.full(U.size, c), dE, g_i, mu, beta)
            th = abs(dE) / 2
            # ramp c (U - th)/(U1 - th) on [th, U1], then c
            U1 = U[0]
            x0, x1 = th / beta, U1 / beta
            ramp_U2 = beta ** 3 * (lower_gamma(3, x1) - lower_gamma(3, x0))   # int U^2 e^-U/beta
            ramp_U1 = beta ** 2 * (lower_gamma(2, x1) - lower_gamma(2, x0))   # int U e^-U/beta
            I = c / (U1 - th) * (ramp_U2 - th * ramp_U1)
            I += c * beta * (U1 + beta) * math.exp(-U1 / beta)
            ref = math.sqrt(8 / (math.pi * mu)) * beta ** -1.5 * math.exp(-dE / (2 * beta)) * I / g_i
            assert abs(k - ref) < 1e-10 * abs(ref), (dE, beta, k, ref)


def test_elastic_constant_is_cross_section_times_mean_speed():
    """sigma(U) = c for all U (threshold at zero, data taken down to U ~ 0)."""
    mu, g_i, c = 2000.0, 1.0, 3.0
    U = np.array([1e-14, 0.001, 0.01, 0.1])
    for beta in (0.001, 0.003):
        k = PP.rate_coefficient(U, np.full(U.size, c), 0.0, g_i, mu, beta)
        assert abs(k - c * math.sqrt(8 * beta / (math.pi * mu))) < 1e-9 * k


def test_linear_cross_section_closed_form():
    mu, g_i = 1000.0, 2.0
    U = np.linspace(0.001, 0.02, 7)
    a, b = 2.0, 150.0
    s_e = a + b * U
    beta, dE = 0.004, 0.0
    k = PP.rate_coefficient(U, s_e, dE, g_i, mu, beta)
    U1, Un = U[0], U[-1]
    # ramp from 0 at U=0 to s_e[0] at U1, spline (exactly linear) to Un, constant after
    ramp = s_e[0] / U1 * beta ** 3 * lower_gamma(3, U1 / beta)
    mid = (a * beta ** 2 * (lower_gamma(2, Un / beta) - lower_gamma(2, U1 / beta))
           + b * beta ** 3 * (lower_gamma(3, Un / beta) - lower_gamma(3, U1 / beta)))
    tail = s_e[-1] * beta * (Un + beta) * math.exp(-Un / beta)
    ref = math.sqrt(8 / (math.pi * mu)) * beta ** -1.5 * (ramp + mid + tail) / g_i
    assert abs(k - ref) < 1e-10 * ref


def test_detailed_balance():
    rng = np.random.default_rng(2)
    L, nE = 4, 10
    U = np.geomspace(2e-4, 0.05, nE)
    g = rng.integers(1, 12, L).astype(float)
    E = np.sort(rng.random(L)) * 0.004
    sigma = rng.random((nE, L, L)) * 20
    sym = PP.symmetrize(sigma, g)
    beta = [0.0003, 0.001, 0.004]
    k = PP.rate_coefficients(U, sym, E, g, 1800.0, beta)
    for t, b in enumerate(beta):
        lhs = g[:, None] * k[t] * np.exp(-E / b)[:, None]
        assert np.max(np.abs(lhs - lhs.T) / np.abs(lhs)) < 1e-12
