"""Cross-section post-processing of the oracle (paper Section III, Eqs. 19-20 and
the rate coefficients built from them).

TEST INFRASTRUCTURE: used only by the tests and the benchmark's CPU baseline.
Plain numpy / scipy, FP64.

  Eq. 19  microscopic reversibility: g' sigma_{n'->n''} = g'' sigma_{n''->n'} with
          g = (2 j1 + 1)(2 j2 + 1) the degeneracy of a level; the diagnostic here is
          the ratio of the two sides.
  Eq. 20  the symmetrised cross section
          sigma~_{n'n''} = (g' sigma_{n'->n''} + g'' sigma_{n''->n'}) / 2.
  rates   k_{n'->n''}(T) from sigma~ integrated over the Maxwell-Boltzmann
          distribution, with a cubic spline through the computed energies.

Readings (the paper defers these details to its ref. 44 -- parity unpinned for
the extrapolation rule):
  * the energies U at which the cross sections are computed are symmetrised
    translational energies (the mean of the initial and final kinetic energies
    of a transition), so that with beta = k_B T
        k_{n'->n''} = (1/g') sqrt(8/(pi mu)) beta^(-3/2) exp(-(E'' - E')/(2 beta))
                      * int_0^inf s(U) U exp(-U/beta) dU,
    which satisfies detailed balance g' k_{n'->n''} exp(-E'/beta) =
    g'' k_{n''->n'} exp(-E''/beta) for any s;
  * s is the natural cubic spline through (U_e, sigma~_e) on [U_1, U_n];
    below U_1 it falls linearly to zero at the threshold U_th = |E'' - E'| / 2
    (zero below U_th; no ramp when U_th >= U_1, the spline then starting at
    U_th); above U_n it stays at sigma~(U_n).
"""
import math

import numpy as np
from scipy import integrate, interpolate


def reversibility_ratio(sigma, g):
    """Eq. 19 left side over right side: g_i sigma[e, i, f] / (g_f sigma[e, f, i]),
    NaN where the right side is zero.  sigma[e, i, f] is sigma_{i->f} at energy e."""
    sigma = np.asarray(sigma, np.float64)
    g = np.asarray(g, np.float64)
    lhs = g[None, :, None] * sigma
    rhs = np.swapaxes(lhs, 1, 2)
    with np.errstate(divide="ignore", invalid="ignore"):
        return np.where(rhs != 0.0, lhs / np.where(rhs != 0.0, rhs, 1.0), np.nan)


def symmetrize(sigma, g):
    """Eq. 20: sigma~[e, i, f] = (g_i sigma_{i->f} + g_f sigma_{f->i}) / 2."""
    sigma = np.asarray(sigma, np.float64)
    g = np.asarray(g, np.float64)
    lhs = g[None, :, None] * sigma
    return 0.5 * (lhs + np.swapaxes(lhs, 1, 2))


def sigma_of_U(U, s_e, U_th):
    """The interpolant s(U) of the readings above, as a callable (vectorised)."""
    U = np.asarray(U, np.float64)
    s_e = np.asarray(s_e, np.float64)
    spl = interpolate.CubicSpline(U, s_e, bc_type="natural")

    def s(x):
        x = np.asarray(x, np.float64)
        out = np.where(x > U[-1], s_e[-1], spl(np.clip(x, U[0], U[-1])))
        if U_th < U[0]:
            out = np.where(x < U[0], s_e[0] * (x - U_th) / (U[0] - U_th), out)
        return np.where(x < U_th, 0.0, out)
    return s


def rate_coefficient(U, s_e, dE, g_i, mu, beta):
    """k_{i->f}(T) for one transition, beta = k_B T, dE = E_f - E_i (atomic units:
    bohr^3 per atomic unit of time).  The Boltzmann factor is taken relative to the
    threshold, exp(-(U - U_th)/beta), and exp(-(U_th + dE/2)/beta) (1 for quenching,
    exp(-dE/beta) for excitation) multiplies the integral, so that nothing over- or
    underflows where the product does not."""
    U_th = abs(dE) / 2.0
    s = sigma_of_U(U, s_e, U_th)
    f = lambda x: float(s(x)) * x * math.exp(-(x - U_th) / beta)
    pts = [p for p in [U_th] + list(U) if p >= U_th]
    total = 0.0
    for a, b in zip(pts[:-1], pts[1:]):
        if b > a:
            total += integrate.quad(f, a, b, epsabs=0.0, epsrel=1e-12, limit=400)[0]
    # constant tail beyond the last energy: s_n int_{U_n}^inf U e^{-(U-U_th)/beta} dU
    Un = max(U[-1], U_th)
    total += s_e[-1] * beta * (Un + beta) * math.exp(-(Un - U_th) / beta)
    return (math.sqrt(8.0 / (math.pi * mu)) * beta ** -1.5
            * math.exp(-(U_th + dE / 2.0) / beta) * total / g_i)


def rate_coefficients(U, sym, E_level, g, mu, beta, pairs=None):
    """k[t, i, f] for every temperature beta[t] and level pair (or only the given
    (i, f) pairs, returned as k[t, p])."""
    U = np.asarray(U, np.float64)
    sym = np.asarray(sym, np.float64)
    L = sym.shape[1]
    if pairs is None:
        out = np.zeros((len(beta), L, L))
        for t, b in enumerate(beta):
            for i in range(L):
                for f in range(L):
                    out[t, i, f] = rate_coefficient(U, sym[:, i, f], E_level[f] - E_level[i],
                                                    g[i], mu, b)
        return out
    out = np.zeros((len(beta), len(pairs)))
    for t, b in enumerate(beta):
        for p, (i, f) in enumerate(pairs):
            out[t, p] = rate_coefficient(U, sym[:, i, f], E_level[f] - E_level[i], g[i], mu, b)
    return out
