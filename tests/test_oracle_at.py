"""Pins of the oracle's decoupled (AT) dynamics.

In AT-MQCT (paper Section III) the quantum equations (Eq. 5) are propagated
along a classical trajectory whose equations (Eqs. 7-10) no longer feel the
quantum state; here the trajectory is driven by a tabulated potential U(R).

  isotropic coupling M(R) = V(R) 1: the Ehrenfest force is -V'(R) |a|^2 and
  the torque vanishes, so AT driven by U = V is the same dynamics          -> driver force sign and
                                                                              magnitude, zero torque
  linearity in the initial state (Ehrenfest is not linear)                 -> no feedback of the
                                                                              quantum state
  trajectory independent of the initial state, bitwise                     -> decoupling
  U-driven classical energy and P_Phi conserved                            -> AT invariants
  U = 0, M = 0: straight line                                              -> centrifugal term
"""
import math

import numpy as np

import oracle
from synth import systems as S
from synth.systems import System


def isotropic_copy(s):
    """The same grid, energies, Coriolis operator and mass, with M(R) = V(R) 1,
    V the average diagonal of the original tables."""
    V = np.real(np.einsum("knn->k", s.M)) / s.N
    M = np.zeros_like(s.M)
    for n in range(s.N):
        M[:, n, n] = V
    return System("iso", s.R_grid, s.E, M, s.jx_row, s.jx_col, s.jx_val, s.mu,
                  s.level_of_channel, s.n_levels), V


def test_at_equals_ehrenfest_for_isotropic_coupling():
    # steps fine enough that the RK4 norm defect (which enters the Ehrenfest
    # force as V'(R) (1 - |a|^2)) stays near 1e-10
    (s,), b = S.config1(n_traj=6, n_steps=6000, jmax=3)
    iso, V = isotropic_copy(s)
    eh = oracle.OracleSystem(iso).propagate(b)
    at = oracle.OracleSystem(iso, driver=V).propagate(b)
    assert np.max(np.abs(eh["norm_err"])) < 1e-9
    assert np.max(np.abs(eh["P"] - at["P"])) < 1e-9
    assert np.max(np.abs(eh["classical"] - at["classical"]) /
                  (1 + np.abs(eh["classical"]))) < 1e-8
    # the molecule turns (Coriolis term on) but exchanges no torque in either form
    assert np.max(np.abs(eh["classical"][:, 5] - at["classical"][:, 5])) < 1e-9
    assert np.max(np.abs(at["classical"][:, 5] - b.b * np.sqrt(2 * s.mu * b.E_coll))) == 0.0
    # with the anisotropic tables the two dynamics differ
    full_eh = oracle.OracleSystem(s).propagate(b)
    full_at = oracle.OracleSystem(s, driver=V).propagate(b)
    assert np.max(np.abs(full_eh["P"] - full_at["P"])) > 1e-6


def test_at_is_linear_in_the_initial_state():
    (s,), b = S.config1(n_traj=3, n_steps=400, jmax=2)
    _, V = isotropic_copy(s)
    N = s.N
    i, j = 4, 6
    al, be = 0.6, 0.8j
    a_sup = np.zeros((b.B, N), complex)
    a_sup[:, i] = al
    a_sup[:, j] = be
    for drv in (V, None):
        o = oracle.OracleSystem(s, driver=drv)
        ri = o.propagate(b, init_channel=np.full(b.B, i))
        rj = o.propagate(b, init_channel=np.full(b.B, j))
        rs = o.propagate(b, a0=a_sup)
        err = np.max(np.abs(rs["a_final"] - (al * ri["a_final"] + be * rj["a_final"])))
        if drv is not None:
            assert err < 1e-12          # AT: a linear map of the initial amplitudes
        else:
            assert err > 1e-6           # Ehrenfest: the mean field makes it nonlinear


def test_at_trajectory_does_not_depend_on_the_initial_state():
    (s,), b = S.config1(n_traj=4, n_steps=300, jmax=3)
    _, V = isotropic_copy(s)
    o = oracle.OracleSystem(s, driver=V)
    r1 = o.propagate(b, init_channel=np.zeros(b.B, np.int32))
    r2 = o.propagate(b, init_channel=np.full(b.B, s.N - 1, np.int32))
    assert np.array_equal(r1["classical"], r2["classical"])
    assert not np.array_equal(r1["P"], r2["P"])


def test_at_invariants():
    """P^2/2mu + P_Phi^2/(2 mu R^2) + U(R) is conserved to the integrator's
    accuracy (a driving force other than -U' -- wrong sign or scale -- breaks
    it at order one), P_Phi exactly, the norm to the RK4 defect."""
    (s,), b = S.config1(n_traj=4, n_steps=4000, jmax=3)
    _, V = isotropic_copy(s)
    r = oracle.OracleSystem(s, driver=V).propagate(b)
    assert np.max(np.abs(r["energy_err"])) < 1e-8
    assert np.max(np.abs(r["angmom_err"])) == 0.0
    assert np.max(np.abs(r["norm_err"])) < 1e-8


def test_at_free_motion_is_a_straight_line():
    (s,), b = S.config1(n_traj=3, n_steps=2000, jmax=1)
    zero = np.zeros(s.K)
    free = System("free", s.R_grid, s.E, np.zeros_like(s.M), s.jx_row, s.jx_col, s.jx_val, s.mu,
                  s.level_of_channel, s.n_levels)
    r = oracle.OracleSystem(free, driver=zero).propagate(b)
    v = np.sqrt(2 * b.E_coll / s.mu)
    T = b.dt * b.n_steps
    s0 = np.sqrt(b.R0 ** 2 - b.b ** 2)
    R_exact = np.sqrt(b.b ** 2 + (s0 - v * T) ** 2)
    Phi_exact = np.arctan2(b.b, s0 - v * T) - np.arctan2(b.b, s0)
    assert np.max(np.abs(r["classical"][:, 0] - R_exact) / R_exact) < 1e-9
    assert np.max(np.abs(r["classical"][:, 2] - Phi_exact)) < 1e-9
