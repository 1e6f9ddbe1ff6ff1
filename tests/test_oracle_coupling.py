"""Pins of the oracle's coupling matrix (Section II, Eq. 17).

  Eq. 17 against Eq. 11: the matrix element as a direct four-dimensional
  quadrature of Psi''* tau_t Psi' (Eq. 3 states, Eq. 13 angular functions) with
  alpha_1 = 0 and the factor 2 pi, the check the paper itself made.  Wigner d
  from Wigner's explicit sum (pinned to spherical harmonics from scipy and to
  the closed-form j = 1 matrix), spherical harmonics from scipy, Gauss-Legendre
  in cos(beta) and equidistant points in the azimuthal angles: exact for these
  band-limited integrands                                              -> every
                                                                          factor,
                                                                          index and
                                                                          phase of Eq. 17
  isotropic term tau_0000 = 1/(2 pi): M = v/(2 pi) 1                   -> normalisation
  Clebsch-Gordan values from tables, closed forms, symmetry,
  orthogonality                                                        -> Racah sum
  real symmetric, zero between different m                             -> Hermiticity of
                                                                          Eq. 6, Eq. 5's
                                                                          m structure
"""
import math

import numpy as np
import pytest
import scipy.special as sp

import oracle
from synth import coupling as C
from synth.angular import clebsch_gordan as cg_exact


# ---------------------------------------------------------------- Clebsch-Gordan

def test_cg_table_values_and_closed_forms():
    table = {(1, 0, 1, 0, 2, 0): math.sqrt(2 / 3), (1, 0, 1, 0, 1, 0): 0.0,
             (1, 0, 1, 0, 0, 0): -1 / math.sqrt(3), (1, 1, 1, -1, 1, 0): 1 / math.sqrt(2),
             (1, 1, 1, -1, 2, 0): 1 / math.sqrt(6), (1, 1, 1, -1, 0, 0): 1 / math.sqrt(3),
             (2, 1, 1, 0, 2, 1): 1 / math.sqrt(6), (2, 0, 1, 1, 3, 1): math.sqrt(2 / 5),
             (1, 1, 1, 0, 2, 1): 1 / math.sqrt(2), (2, 2, 2, -2, 0, 0): 1 / math.sqrt(5)}
    for args, v in table.items():
        assert abs(oracle.cg(*args) - v) < 1e-15, args
    for j in range(0, 9):
        for m in range(-j, j + 1):
            assert abs(oracle.cg(j, m, j, -m, 0, 0) - (-1) ** (j - m) / math.sqrt(2 * j + 1)) < 1e-15
        for j2 in range(0, 6):
            assert abs(oracle.cg(j, j, j2, j2, j + j2, j + j2) - 1.0) < 1e-15


def test_cg_symmetry_and_orthogonality():
    for j1 in range(0, 6):
        for j2 in range(0, 5):
            for M in range(-(j1 + j2), j1 + j2 + 1):
                Js = [J for J in range(abs(j1 - j2), j1 + j2 + 1) if abs(M) <= J]
                ms = [m1 for m1 in range(-j1, j1 + 1) if abs(M - m1) <= j2]
                U = np.array([[oracle.cg(j1, m1, j2, M - m1, J, M) for m1 in ms] for J in Js])
                assert np.max(np.abs(U @ U.T - np.eye(len(Js)))) < 1e-14
                for J in Js:
                    for m1 in ms:
                        a = oracle.cg(j1, m1, j2, M - m1, J, M)
                        assert abs(a - (-1) ** (j1 + j2 - J) * oracle.cg(j2, M - m1, j1, m1, J, M)) < 1e-15
    # larger arguments against exact rational arithmetic
    rng = np.random.default_rng(4)
    for _ in range(200):
        j1, j2 = rng.integers(0, 16, 2)
        J = rng.integers(abs(j1 - j2), j1 + j2 + 1)
        m1 = rng.integers(-j1, j1 + 1)
        M = rng.integers(-J, J + 1)
        args = (int(j1), int(m1), int(j2), int(M - m1), int(J), int(M))
        assert abs(oracle.cg(*args) - cg_exact(*args)) < 1e-14


# ---------------------------------------------------------------- Wigner functions

def wigner_d(j, mp, m, beta):
    """d^j_{m' m}(beta), Wigner's explicit sum."""
    f = math.factorial
    c, s = np.cos(beta / 2), np.sin(beta / 2)
    out = np.zeros_like(beta, dtype=np.float64)
    for k in range(max(0, m - mp), min(j + m, j - mp) + 1):
        num = (-1) ** (mp - m + k) * math.sqrt(f(j + mp) * f(j - mp) * f(j + m) * f(j - m))
        den = f(j + m - k) * f(k) * f(mp - m + k) * f(j - mp - k)
        out = out + num / den * c ** (2 * j + m - mp - 2 * k) * s ** (mp - m + 2 * k)
    return out


def D_conj(j, mp, m, alpha, beta, gamma):
    """D^{j*}_{m' m}(alpha, beta, gamma), D = exp(-i m' alpha) d(beta) exp(-i m gamma)."""
    return np.exp(1j * mp * alpha) * wigner_d(j, mp, m, beta) * np.exp(1j * m * gamma)


def Y(l, m, beta, alpha):
    return sp.sph_harm_y(l, m, beta, alpha)


def test_wigner_d_pins():
    beta = np.linspace(0.0, math.pi, 7)
    c, s = np.cos(beta), np.sin(beta)
    closed = {(1, 1): (1 + c) / 2, (1, 0): -s / math.sqrt(2), (1, -1): (1 - c) / 2,
              (0, 0): c, (0, 1): s / math.sqrt(2), (-1, -1): (1 + c) / 2}
    for (mp, m), v in closed.items():
        assert np.max(np.abs(wigner_d(1, mp, m, beta) - v)) < 1e-15
    for l in range(0, 6):
        for m in range(-l, l + 1):
            y = Y(l, m, beta, 0.0)
            assert np.max(np.abs(wigner_d(l, m, 0, beta) - math.sqrt(4 * math.pi / (2 * l + 1)) * y)) < 1e-14


# ---------------------------------------------------------------- Eq. 11 quadrature

def quadrature_matrices(basis, terms, n_beta=12, n_phi=16):
    """2 pi * integral over (beta1, gamma1, alpha2, beta2) of Psi''* tau_t Psi' (Eq. 11).

    Setting alpha_1 = 0 is exact only when the integrand depends on alpha_2 -
    alpha_1 alone, i.e. between states of the same m; elements between different m
    are left at zero (the full integral over alpha_1 removes them)."""
    x, wx = np.polynomial.legendre.leggauss(n_beta)
    beta = np.arccos(x)
    phi = 2 * math.pi * np.arange(n_phi) / n_phi
    wphi = np.full(n_phi, 2 * math.pi / n_phi)
    B1, G1, A2, B2 = np.meshgrid(beta, phi, phi, beta, indexing="ij")
    W = (wx[:, None, None, None] * wphi[None, :, None, None] * wphi[None, None, :, None]
         * wx[None, None, None, :]).ravel()
    B1, G1, A2, B2 = (a.ravel() for a in (B1, G1, A2, B2))
    N = basis.N
    Psi = np.zeros((N, B1.size), complex)
    for n in range(N):
        j, m, j2 = int(basis.j[n]), int(basis.m[n]), int(basis.j2[n])
        r = int(basis.rot1[n])
        j1 = int(basis.rot1_j[r])
        b = basis.b[r]
        acc = np.zeros(B1.size, complex)
        for m1 in range(-j1, j1 + 1):
            c = cg_exact(j1, m1, j2, m - m1, j, m)
            if c == 0.0:
                continue
            top = sum(b[k + j1] * D_conj(j1, m1, k, 0.0, B1, G1) for k in range(-j1, j1 + 1))
            acc += c * top * Y(j2, m - m1, B2, A2)
        Psi[n] = math.sqrt((2 * j1 + 1) / (8 * math.pi ** 2)) * acc
    out = []
    for (l1, mu1, l2, l) in terms:
        s = (-1) ** (l1 + mu1 + l2 + l)
        tau = np.zeros(B1.size, complex)
        for eta in range(-min(l1, l2), min(l1, l2) + 1):
            c = cg_exact(l1, eta, l2, -eta, l, 0)
            if c == 0.0:
                continue
            tau += c * (D_conj(l1, eta, mu1, 0.0, B1, G1) + s * D_conj(l1, eta, -mu1, 0.0, B1, G1)) \
                * Y(l2, -eta, B2, A2)
        tau *= math.sqrt((2 * l1 + 1) / (4 * math.pi))
        out.append(2 * math.pi * (np.conj(Psi) * (W * tau)[None, :]) @ Psi.T)
    same_m = basis.m[:, None] == basis.m[None, :]
    return np.array(out) * same_m[None]


def all_terms(l1max, l2max):
    return [(l1, mu1, l2, l) for l1 in range(l1max + 1) for mu1 in range(l1 + 1)
            for l2 in range(l2max + 1) for l in range(abs(l1 - l2), l1 + l2 + 1)]


@pytest.mark.parametrize("m_values", [(-1, 0, 2), (1, -2, 3)])
def test_eq17_matches_direct_quadrature_eq11(m_values):
    basis = C.top_rotor_basis(2, (0, 1, 2), m_values=m_values)
    terms = all_terms(3, 2)
    arr = [np.array([t[i] for t in terms]) for i in range(4)]
    G = oracle.coupling_angular(basis, *arr)
    Q = quadrature_matrices(basis, terms)
    # the expansion functions are real, so Eq. 11 gives real matrices
    assert np.max(np.abs(Q.imag)) < 1e-13
    err = np.max(np.abs(G - Q.real))
    scale = np.max(np.abs(Q.real))
    print("Eq. 17 vs Eq. 11: %d terms, N = %d, max |diff| %.2e of %.2e" % (len(terms), basis.N, err, scale))
    assert err < 1e-13 * max(scale, 1.0)
    # the check covers couplings between different rotor-1 states and different j2
    cross = (basis.rot1[:, None] != basis.rot1[None, :]) & (basis.j2[:, None] != basis.j2[None, :])
    assert np.count_nonzero(np.abs(G[:, cross]) > 1e-3) > 1000


def test_isotropic_term_and_structure():
    basis = C.top_rotor_basis(3, (0, 2))
    terms = [(0, 0, 0, 0), (2, 2, 2, 2), (3, 2, 0, 3), (4, 0, 2, 2), (2, 0, 2, 4)]
    arr = [np.array([t[i] for t in terms]) for i in range(4)]
    G = oracle.coupling_angular(basis, *arr)
    assert np.max(np.abs(G[0] - np.eye(basis.N) / (2 * math.pi))) < 1e-15
    same_m = basis.m[:, None] == basis.m[None, :]
    for g in G:
        assert np.max(np.abs(g - g.T)) < 1e-15
        assert np.all(g[~same_m] == 0.0)
