"""Checks of the seeded input generators (not of the propagator)."""
import math

import numpy as np
from scipy.special import roots_legendre, sph_harm_y, eval_legendre

from synth import angular as A, systems as S, units as U


def test_gaunt_against_quadrature():
    """<j'' m | P_lam | j' m> (one-rotor case of Section II, Eq. 15) vs Gauss-Legendre."""
    x, w = roots_legendre(40)
    th = np.arccos(x)
    for (j2, j1, lam, m) in [(2, 0, 2, 0), (3, 1, 2, 1), (4, 2, 2, -2), (3, 3, 4, 2), (5, 1, 4, 0),
                             (2, 1, 1, 1)]:
        y2 = sph_harm_y(j2, m, th, 0.0)
        y1 = sph_harm_y(j1, m, th, 0.0)
        quad = 2 * math.pi * np.sum(w * np.conj(y2) * eval_legendre(lam, x) * y1).real
        assert abs(A.legendre_matrix_element(j2, j1, lam, m) - quad) < 1e-13


def test_gaunt_selection_rule():
    for j1 in range(4):
        for j2 in range(4):
            for lam in range(5):
                if (j1 + j2 + lam) % 2 == 1:
                    assert A.legendre_matrix_element(j2, j1, lam, 0) == 0.0


def test_asymmetric_top_sum_rule_and_prolate_limit():
    Arot, Brot, Crot = 27.0, 14.5, 9.3
    for j in range(9):
        lev = A.asymmetric_top_levels(j, Arot, Brot, Crot)
        assert abs(lev.sum() - (2 * j + 1) * j * (j + 1) * (Arot + Brot + Crot) / 3) < 1e-10
    lev = A.asymmetric_top_levels(4, 10.0, 3.0, 3.0)
    ref = sorted(3.0 * 20 + 7.0 * k * k for k in range(-4, 5))
    assert np.allclose(lev, ref, atol=1e-10)


def test_clebsch_gordan_orthonormality():
    j1, j2 = 2, 3
    for J in range(1, 6):
        for M in range(-J, J + 1):
            s = sum(A.clebsch_gordan(j1, m1, j2, M - m1, J, M) ** 2 for m1 in range(-j1, j1 + 1))
            assert abs(s - 1.0) < 1e-14


def test_config_shapes_and_hermiticity():
    (s1,), b1 = S.config1()
    assert s1.N == 49 and s1.K == 200 and b1.B == 64 and np.all(b1.n_steps == 2000)
    assert np.array_equal(s1.M, np.swapaxes(s1.M, 1, 2))
    (s4,), b4 = S.config4(n_traj=16)
    assert s4.N == 256 and s4.theta.shape == (96,)
    assert np.allclose(S.parametric_tables(s4, s4.theta), s4.M, atol=1e-18)
    (s2,), b2 = S.config2(n_traj=8, jmax=3)
    assert s2.N == 84 and np.iscomplexobj(s2.M)
    assert np.array_equal(s2.M, np.conj(np.swapaxes(s2.M, 1, 2)))
    # cfg 2 full size is N = 969 (j <= 8, all tau and m)
    assert sum((2 * j + 1) ** 2 for j in range(9)) == 969
    # coupling magnitudes in the paper's range (1e-4 .. 1e2 cm^-1 and a repulsive wall)
    k3 = np.argmin(np.abs(s1.labels["R_ang"] - 3.0))
    assert 1e-4 < np.max(np.abs(U.hartree_to_cm(s1.M[k3] - np.diag(np.diag(s1.M[k3]))))) < 1e3


def test_seeded_reproducibility():
    (a,), ba = S.config1(n_traj=8)
    (b,), bb = S.config1(n_traj=8)
    assert np.array_equal(a.M, b.M) and np.array_equal(ba.b, bb.b)
