"""Angular-momentum coefficients used to build synthetic coupling tables.

These are input-construction helpers: Clebsch-Gordan coefficients from the
Racah closed form, the Gaunt integral of three spherical harmonics (Section II,
Eq. 15) and rigid-rotor energies.  Nothing here propagates a trajectory.
"""
from fractions import Fraction
from functools import lru_cache
import math

import numpy as np


@lru_cache(maxsize=None)
def _fact(n):
    return math.factorial(n)


@lru_cache(maxsize=None)
def clebsch_gordan(j1, m1, j2, m2, J, M):
    """<j1 m1 j2 m2 | J M> for integer angular momenta (Racah's closed form)."""
    if m1 + m2 != M:
        return 0.0
    if J < abs(j1 - j2) or J > j1 + j2:
        return 0.0
    if abs(m1) > j1 or abs(m2) > j2 or abs(M) > J:
        return 0.0
    pre = Fraction((2 * J + 1) * _fact(J + j1 - j2) * _fact(J - j1 + j2) * _fact(j1 + j2 - J),
                   _fact(j1 + j2 + J + 1))
    pre *= (_fact(J + M) * _fact(J - M) * _fact(j1 - m1) * _fact(j1 + m1)
            * _fact(j2 - m2) * _fact(j2 + m2))
    s = Fraction(0)
    kmin = max(0, j2 - J - m1, j1 - J + m2)
    kmax = min(j1 + j2 - J, j1 - m1, j2 + m2)
    for k in range(kmin, kmax + 1):
        den = (_fact(k) * _fact(j1 + j2 - J - k) * _fact(j1 - m1 - k) * _fact(j2 + m2 - k)
               * _fact(J - j2 + m1 + k) * _fact(J - j1 - m2 + k))
        s += Fraction((-1) ** k, den)
    if s == 0:
        return 0.0
    sign = 1.0 if s > 0 else -1.0
    # sqrt(pre) * s, evaluated as sqrt(pre * s^2) to keep the rational part exact
    return sign * math.sqrt(pre * s * s)


def gaunt(l3, m3, l2, m2, l1, m1):
    """<Y_{l3 m3} | Y_{l2 m2} | Y_{l1 m1}> as in Section II, Eq. 15."""
    return (math.sqrt((2 * l1 + 1) * (2 * l2 + 1) / (4.0 * math.pi * (2 * l3 + 1)))
            * clebsch_gordan(l1, 0, l2, 0, l3, 0) * clebsch_gordan(l1, m1, l2, m2, l3, m3))


def legendre_matrix_element(j2, j1, lam, m):
    """<j2 m | P_lam(cos theta) | j1 m>: the one-rotor special case of Eq. 15."""
    return (math.sqrt((2 * j1 + 1) / (2 * j2 + 1))
            * clebsch_gordan(j1, 0, lam, 0, j2, 0) * clebsch_gordan(j1, m, lam, 0, j2, m))


def asymmetric_top_levels(j, A, B, C):
    """Eigenvalues (ascending, tau = -j..j) of A Ja^2 + B Jb^2 + C Jc^2 for one j.

    Symmetric-top basis |j k> with k along the a axis (Section II, Eq. 1): the
    diagonal is (B+C)/2 (j(j+1) - k^2) + A k^2 and k couples to k+-2 with
    (B-C)/4 sqrt[(j(j+1) - k(k+1)) (j(j+1) - (k+1)(k+2))].
    """
    n = 2 * j + 1
    H = np.zeros((n, n))
    jj = j * (j + 1)
    for i, k in enumerate(range(-j, j + 1)):
        H[i, i] = 0.5 * (B + C) * (jj - k * k) + A * k * k
        if k + 2 <= j:
            off = 0.25 * (B - C) * math.sqrt((jj - k * (k + 1)) * (jj - (k + 1) * (k + 2)))
            H[i, i + 2] = off
            H[i + 2, i] = off
    return np.linalg.eigvalsh(H)


def asymmetric_top_states(j, A, B, C):
    """Energies (ascending, tau = -j..j) and eigenvectors of the rigid asymmetric top
    for one j, in the basis of Section II, Eq. 1 (coefficients b_k, k = -j..j).

    Same Hamiltonian matrix as asymmetric_top_levels.  Row tau + j of the returned
    array holds b_k of level tau; each vector is normalised and its largest
    component made positive so that the phases are reproducible.
    """
    n = 2 * j + 1
    H = np.zeros((n, n))
    jj = j * (j + 1)
    for i, k in enumerate(range(-j, j + 1)):
        H[i, i] = 0.5 * (B + C) * (jj - k * k) + A * k * k
        if k + 2 <= j:
            off = 0.25 * (B - C) * math.sqrt((jj - k * (k + 1)) * (jj - (k + 1) * (k + 2)))
            H[i, i + 2] = off
            H[i + 2, i] = off
    E, V = np.linalg.eigh(H)
    b = V.T.copy()
    for r in range(n):
        big = int(np.argmax(np.abs(b[r])))
        if b[r, big] < 0:
            b[r] = -b[r]
    return E, b


def jx_block(j):
    """Rows, cols, values of J_x on |j m>, m = -j..j (indices local to the block).

    <m|J_x|m-1> = sqrt(j(j+1) - m(m-1))/2 and <m|J_x|m+1> = sqrt(j(j+1) - m(m+1))/2,
    the Coriolis coefficients of Section II, Eq. 5.
    """
    rows, cols, vals = [], [], []
    jj = j * (j + 1)
    for i, m in enumerate(range(-j, j + 1)):
        if m - 1 >= -j:
            rows.append(i); cols.append(i - 1); vals.append(0.5 * math.sqrt(jj - m * (m - 1)))
        if m + 1 <= j:
            rows.append(i); cols.append(i + 1); vals.append(0.5 * math.sqrt(jj - m * (m + 1)))
    return rows, cols, vals
