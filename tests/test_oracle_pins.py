"""Pins of the FP64 oracle against closed forms, invariants and library routines.

Each test ties one part of the oracle to something other than itself, so that a
dropped term, a wrong sign, a wrong index or a transposed operand fails at least
one of them:

  spline (scipy natural CubicSpline, linear exactness, off-grid rule)  -> table interpolation
  Rabi two-level closed form                                             -> coupling term, phases
  frozen trajectory vs scipy expm, complex Hermitian, N = 5              -> phase sign, orientation of M
  free straight line + Wigner small-d populations                       -> classical Eqs. 7-8, centrifugal
                                                                           term, Coriolis magnitude
  energy conservation                                                    -> Coriolis sign, force sign, M'
  P_Phi - <J_x> conservation                                             -> torque (Eq. 10)
  norm conservation                                                      -> Hermitian generator
  m-reflection symmetry                                                  -> J_x indices
  RK4 order and DOP853 comparison                                        -> the RK4 stepper
  scipy RK45 on the oracle's right-hand side (same tableau and controller) -> DP5 weights, error
                                                                           norm, step-factor rule,
                                                                           starting step
  h^5 scaling of one attempt's embedded error estimate on a' = -iVa      -> DP5 error weights
  dual-number derivative vs central differences                          -> forward mode
  Monte-Carlo estimator closed form and the l_max = k b_max relation     -> cross sections, initial state
"""
import math

import numpy as np
import pytest
from scipy.interpolate import CubicSpline
from scipy.integrate import solve_ivp
from scipy.linalg import expm

import oracle
from synth import systems as S, units as U
from synth.systems import System


def make_system(R, E, M, jx=None, mu=1000.0):
    N = len(E)
    if jx is None:
        jr = jc = np.zeros(0, np.int32); jv = np.zeros(0)
    else:
        jr, jc, jv = (np.asarray(jx[0], np.int32), np.asarray(jx[1], np.int32),
                      np.asarray(jx[2], np.float64))
    return System("test", np.asarray(R, float), np.asarray(E, float), M, jr, jc, jv, float(mu),
                  np.arange(N, dtype=np.int32), N)


# ------------------------------------------------------------------ spline

def test_spline_matches_scipy_natural():
    rng = np.random.default_rng(1)
    x = np.cumsum(rng.uniform(0.1, 0.6, 40)) + 2.0
    y = rng.standard_normal((40, 3))
    y2 = oracle.spline_prepare(x, y)
    for r in rng.uniform(x[0], x[-1], 50):
        v, d, below = oracle.spline_eval(x, y, y2, r)
        assert not below
        for c in range(3):
            cs = CubicSpline(x, y[:, c], bc_type="natural")
            assert abs(v[c] - cs(r)) <= 1e-12 * (1 + abs(cs(r)))
            assert abs(d[c] - cs(r, 1)) <= 1e-11 * (1 + abs(cs(r, 1)))
    cs = CubicSpline(x, y[:, 0], bc_type="natural")
    assert np.allclose(y2[:, 0], cs(x, 2), atol=1e-11)


def test_spline_exact_on_linear_and_offgrid_rule():
    x = np.linspace(3.0, 30.0, 25)
    y = (2.5 * x - 1.0)[:, None]
    y2 = oracle.spline_prepare(x, y)
    assert np.max(np.abs(y2)) < 1e-12
    v, d, below = oracle.spline_eval(x, y, y2, 7.3)
    assert abs(v[0] - (2.5 * 7.3 - 1.0)) < 1e-12 and abs(d[0] - 2.5) < 1e-12 and not below
    # above the last knot: value held, slope zero
    v, d, below = oracle.spline_eval(x, y, y2, 31.0)
    assert v[0] == pytest.approx(2.5 * 30.0 - 1.0, abs=1e-12) and d[0] == 0.0 and not below
    # below the first knot: linear continuation with the end slope, flagged
    yq = (x ** 2)[:, None]
    y2q = oracle.spline_prepare(x, yq)
    v0, d0, _ = oracle.spline_eval(x, yq, y2q, 3.0)
    v, d, below = oracle.spline_eval(x, yq, y2q, 2.5)
    assert below and d[0] == pytest.approx(d0[0], abs=1e-13)
    assert v[0] == pytest.approx(v0[0] - 0.5 * d0[0], abs=1e-12)


# ------------------------------------------------------------------ closed forms

def test_rabi_two_level():
    """N = 2, constant coupling V: P_2(t) = (4V^2/Omega^2) sin^2(Omega t/2)."""
    Delta, V = 0.02, 0.015
    R = np.linspace(4.0, 40.0, 30)
    M = np.zeros((30, 2, 2)); M[:, 0, 1] = M[:, 1, 0] = V
    o = oracle.OracleSystem(make_system(R, [0.0, Delta], M))
    Om = math.sqrt(Delta ** 2 + 4 * V ** 2)
    T = 700.0
    for n in (2000, 4000):
        out = o.propagate(init_channel=[0], E_coll=[1e-3], b=[0.0], R0=[30.0], dt=[T / n],
                          n_steps=[n])
        exact = 4 * V ** 2 / Om ** 2 * math.sin(Om * T / 2) ** 2
        err = abs(out["P"][0, 1] - exact)
    assert err < 1e-10
    assert abs(out["P"][0].sum() - 1) < 1e-12


def test_frozen_trajectory_matches_expm():
    """Infinite mass freezes R: a(t) = e^{iEt} expm(-i(E + M(R0))t) a0 (phase convention)."""
    rng = np.random.default_rng(7)
    N, K = 5, 20
    R = np.linspace(4.0, 24.0, K)
    E = np.sort(rng.uniform(0.0, 0.03, N))
    X = rng.standard_normal((K, N, N)) + 1j * rng.standard_normal((K, N, N))
    M = 0.01 * (X + np.conj(np.swapaxes(X, 1, 2))) / 2
    jx = ([0, 1], [1, 0], [0.7, 0.7])
    o = oracle.OracleSystem(make_system(R, E, M, jx=jx, mu=1e30))
    k0 = 9
    T, n = 300.0, 6000
    out = o.propagate(init_channel=[1], E_coll=[1e-3], b=[0.0], R0=[R[k0]], dt=[T / n],
                      n_steps=[n])
    b0 = np.zeros(N, complex); b0[1] = 1
    bT = expm(-1j * (np.diag(E) + M[k0]) * T) @ b0
    aT = np.exp(1j * E * T) * bT
    assert np.max(np.abs(out["a_final"][0] - aT)) < 1e-10
    # the transposed coupling (a plausible slip) gives a visibly different answer
    bT_wrong = expm(-1j * (np.diag(E) + M[k0].T) * T) @ b0
    assert np.max(np.abs(np.exp(1j * E * T) * bT_wrong - aT)) > 1e-3


def wigner_small_d(j, mp, m, beta):
    """Textbook closed form of d^j_{m' m}(beta)."""
    f = math.factorial
    s = 0.0
    for k in range(0, 2 * j + 1):
        if j + m - k < 0 or j - k - mp < 0 or k - m + mp < 0:
            continue
        num = (-1) ** (k - m + mp) * math.sqrt(f(j + mp) * f(j - mp) * f(j + m) * f(j - m))
        den = f(j + m - k) * f(k) * f(j - k - mp) * f(k - m + mp)
        s += num / den * math.cos(beta / 2) ** (2 * j - 2 * k + m - mp) \
            * math.sin(beta / 2) ** (2 * k - m + mp)
    return s


def test_zero_coupling_straight_line_and_wigner_rotation():
    """M = 0: free straight-line motion; J_x turns the m populations by Phi(t)."""
    (s1,), _ = S.config1(n_traj=1, jmax=3)
    s = make_system(s1.R_grid, s1.E, np.zeros_like(s1.M), jx=(s1.jx_row, s1.jx_col, s1.jx_val),
                    mu=s1.mu)
    o = oracle.OracleSystem(s)
    U_ = U.cm_to_hartree(500.0)
    bpar, R0 = 6.0, s.R_grid[-1]
    v = math.sqrt(2 * U_ / s.mu)
    s0 = math.sqrt(R0 ** 2 - bpar ** 2)
    T = 1.3 * s0 / v
    ch = 9 + 2          # j = 3, m = -1 (channels ordered j, m)
    assert s1.labels["j"][ch] == 3 and s1.labels["m"][ch] == -1
    out = o.propagate(init_channel=[ch], E_coll=[U_], b=[bpar], R0=[R0], dt=[T / 4000],
                      n_steps=[4000])
    Rex = math.sqrt(bpar ** 2 + (s0 - v * T) ** 2)
    Phex = math.atan2(bpar, s0 - v * T) - math.atan2(bpar, s0)
    R, Ph = out["classical"][0, 0], out["classical"][0, 2]
    assert abs(R - Rex) < 1e-9 * Rex
    assert abs(Ph - Phex) < 1e-10
    assert out["classical"][0, 1] == math.pi / 2 and out["classical"][0, 4] == 0.0
    P = out["P"][0]
    for idx in range(9, 16):
        mpp = s1.labels["m"][idx]
        assert abs(P[idx] - wigner_small_d(3, mpp, -1, Phex) ** 2) < 1e-10
    assert P[:9].sum() < 1e-28


# ------------------------------------------------------------------ invariants

def _cfg1_small_dt(n_traj=6, n_steps=20000, jmax=6):
    (s,), b = S.config1(n_traj=n_traj, n_steps=n_steps, jmax=jmax)
    return s, b


@pytest.fixture(scope="module")
def cfg1_fine():
    s, b = _cfg1_small_dt()
    o = oracle.OracleSystem(s)
    return s, b, o.propagate(b)


def test_norm_energy_angular_momentum(cfg1_fine):
    s, b, out = cfg1_fine
    assert np.max(np.abs(out["norm_err"])) < 1e-10
    assert np.max(np.abs(out["energy_err"])) < 1e-9
    assert np.max(np.abs(out["angmom_err"])) < 1e-10
    # the collisions are not trivial: some population leaves the initial level
    lev = s.level_of_channel
    inel = [out["P"][i][lev != b.init_level[i]].sum() for i in range(b.B)]
    assert max(inel) > 1e-3


def test_energy_pins_coriolis_sign():
    """A planted sign slip (+i Phidot J_x in Eq. 5, torque unchanged) breaks energy conservation."""
    s, b = _cfg1_small_dt(n_traj=6, n_steps=20000)
    good = oracle.OracleSystem(s).propagate(b)
    bad = oracle.OracleSystem(s, plant_coriolis_flip=True).propagate(b)
    assert np.max(np.abs(good["energy_err"])) < 1e-9
    assert np.max(np.abs(bad["energy_err"])) > 1e-6


def test_m_reflection_symmetry():
    (s,), b = S.config1(n_traj=4, n_steps=1500, jmax=4)
    o = oracle.OracleSystem(s)
    j, m = s.labels["j"], s.labels["m"]
    idx = {(jj, mm): i for i, (jj, mm) in enumerate(zip(j, m))}
    ch = np.array([idx[(2, 1)]] * 4, np.int32)
    chr_ = np.array([idx[(2, -1)]] * 4, np.int32)
    p1 = o.propagate(b, init_channel=ch)["P"]
    p2 = o.propagate(b, init_channel=chr_)["P"]
    mirror = np.array([idx[(jj, -mm)] for jj, mm in zip(j, m)])
    assert np.max(np.abs(p1 - p2[:, mirror])) < 1e-12
    assert np.max(np.abs(p1 - p2)) > 1e-6      # the reflection is not trivial


def test_literal_phases_equal_factorised():
    (s,), b = S.config1(n_traj=3, n_steps=400, jmax=3)
    p1 = oracle.OracleSystem(s).propagate(b)["a_final"]
    p2 = oracle.OracleSystem(s, literal_phase=True).propagate(b)["a_final"]
    assert np.max(np.abs(p1 - p2)) < 1e-12


# ------------------------------------------------------------------ integrators

def test_rk4_fourth_order():
    (s,), b = S.config1(n_traj=1, n_steps=1, jmax=3)
    o = oracle.OracleSystem(s)
    T = 40000.0
    ref = o.propagate(b, dt=[T / 32000], n_steps=[32000])["a_final"][0]
    errs = []
    for n in (200, 400, 800):
        a = o.propagate(b, dt=[T / n], n_steps=[n])["a_final"][0]
        errs.append(np.max(np.abs(a - ref)))
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 13.0 < r1 < 19.0 and 13.0 < r2 < 19.0, errs


def _state0(o, ch, E_coll, bpar, R0):
    N = o.N
    y = np.zeros(2 * N + 6)
    y[2 * ch] = 1.0
    k = math.sqrt(2 * o.mu * E_coll)
    y[2 * N:] = [R0, math.pi / 2, 0.0, -math.sqrt(k ** 2 - (bpar * k) ** 2 / R0 ** 2), 0.0,
                 bpar * k]
    return y


def test_rk4_against_dop853():
    """An independent integrator (scipy DOP853) on the oracle's right-hand side
    pins the fixed-step RK4 stepper."""
    (s,), b = S.config1(n_traj=1, n_steps=1, jmax=2)
    o = oracle.OracleSystem(s)
    E_coll, bpar, R0 = b.E_coll[0], 3.0, s.R_grid[-1]
    y0 = _state0(o, int(b.init_channel[0]), E_coll, bpar, R0)
    T = 60000.0
    sol = solve_ivp(lambda t, y: o.rhs(t, y)[0], (0.0, T), y0, method="DOP853", rtol=1e-13,
                    atol=1e-13)
    yT = sol.y[:, -1]
    out = o.propagate(init_channel=b.init_channel, E_coll=[E_coll], b=[bpar], R0=[R0],
                      dt=[T / 40000], n_steps=[40000])
    N = o.N
    aT = yT[:2 * N:2] + 1j * yT[1:2 * N:2]
    # The splined coupling is only C^2 in R, so across every knot the eighth-order
    # DOP853 loses order; at rtol 1e-13 its own global error is a few 1e-9, while
    # RK4 at this step is converged to ~1e-12.  A wrong RK4 weight would show ~1e-3.
    assert np.max(np.abs(out["a_final"][0] - aT)) < 2e-8
    assert np.max(np.abs(out["classical"][0] - yT[2 * N:]) / (1 + np.abs(yT[2 * N:]))) < 2e-8


def _scipy_rk45(o, y0, rtol, atol, until_exit=None, n_accepted=None):
    """scipy's RK45 (the Dormand-Prince 5(4) pair with first-same-as-last, the RMS
    norm scaled by atol + rtol max(|y|, |y_new|), the factor 0.9 err^-1/5 bounded by
    0.2 below, no growth right after a rejection, the Hairer-Norsett-Wanner starting
    step) with its growth bound set to 5, stepping the oracle's right-hand side.
    Returns (accepted, rejected, t, y)."""
    import scipy.integrate._ivp.rk as rk
    from scipy.integrate import RK45
    nfev = [0]

    def f(t, y):
        nfev[0] += 1
        return o.rhs(t, y)[0]

    old = rk.MAX_FACTOR
    rk.MAX_FACTOR = 5.0
    try:
        sol = RK45(f, 0.0, y0.copy(), t_bound=1e15, rtol=rtol, atol=atol)
        n = 0
        while True:
            sol.step()
            n += 1
            if n_accepted is not None and n == n_accepted:
                break
            if until_exit is not None and sol.y[2 * o.N] >= until_exit and sol.y[2 * o.N + 3] > 0:
                break
    finally:
        rk.MAX_FACTOR = old
    # two evaluations before the first attempt (f(t0, y0) and the starting-step
    # probe), then six per attempt
    attempts = (nfev[0] - 2) // 6
    assert nfev[0] == 2 + 6 * attempts
    return n, attempts - n, sol.t, sol.y


@pytest.mark.parametrize("bpar", [3.0, 8.0])
def test_dp5_controller_matches_scipy_rk45(bpar):
    """The oracle's adaptive stepper against scipy's RK45 on the same right-hand
    side: the same accepted and rejected step counts over a whole collision (and
    over the first 40 accepted steps, stopped by the accepted-step limit), the same
    end time and state.  The decisions agree one by one only if the error weights,
    the norm, the factor rule and the starting step all agree; the times then differ
    only by rounding of the error estimates (amplified along the step sequence)."""
    (s,), b = S.config1(n_traj=1, n_steps=1, jmax=2)
    o = oracle.OracleSystem(s)
    N = o.N
    E_coll, R0 = b.E_coll[0], s.R_grid[-1]
    ch = int(b.init_channel[0])
    y0 = _state0(o, ch, E_coll, bpar, R0)
    kw = dict(init_channel=[ch], E_coll=[E_coll], b=[bpar], R0=[R0], method="dp5", rtol=1e-8,
              atol=1e-8)
    full = o.propagate(**kw)
    assert full["status"][0] & oracle.STATUS["EXITED"]
    n, rej, t, y = _scipy_rk45(o, y0, 1e-8, 1e-8, until_exit=R0)
    assert rej > 5, rej             # the rejection branch is exercised
    assert (int(full["steps"][0]), int(full["rejects"][0])) == (n, rej)
    assert abs(full["t_final"][0] - t) <= 1e-7 * t
    a = y[:2 * N:2] + 1j * y[1:2 * N:2]
    assert np.max(np.abs(full["a_final"][0] - a)) < 1e-7
    assert np.max(np.abs(full["classical"][0] - y[2 * N:]) / (1 + np.abs(y[2 * N:]))) < 1e-7
    part = o.propagate(max_steps=40, **kw)
    n, rej, t, y = _scipy_rk45(o, y0, 1e-8, 1e-8, n_accepted=40)
    assert part["status"][0] & oracle.STATUS["MAX_STEPS"]
    assert (int(part["steps"][0]), int(part["rejects"][0])) == (n, rej)
    assert abs(part["t_final"][0] - t) <= 1e-9 * t
    a = y[:2 * N:2] + 1j * y[1:2 * N:2]
    assert np.max(np.abs(part["a_final"][0] - a)) < 1e-8


def test_dp5_embedded_error_is_fifth_order():
    """One attempt on a' = -i V a (one channel, constant coupling, head-on free
    flight: the classical part is linear in t and integrated exactly): the embedded
    estimate is the difference of a fifth- and a fourth-order solution, so it scales
    as h^5 -- a wrong error weight breaks an order condition and changes the power."""
    V = 0.01
    R = np.linspace(3.0, 40.0, 12)
    o = oracle.OracleSystem(make_system(R, [0.0], np.full((12, 1, 1), V), mu=2000.0))
    y0 = np.zeros(8)
    y0[0] = 1.0
    y0[2:] = [20.0, math.pi / 2, 0.0, -5.0, 0.0, 0.0]
    errs = [o.dp5_error(0.0, y0, h, 1e-8, 1e-8)[0] for h in (4.0, 2.0, 1.0)]
    r1, r2 = errs[0] / errs[1], errs[1] / errs[2]
    assert 30.0 < r1 < 34.0 and 31.0 < r2 < 33.0, errs
    # the fifth-order solution itself is the exponential to O(h^6)
    en, yn = o.dp5_error(0.0, y0, 1.0, 1e-8, 1e-8)
    assert abs(complex(yn[0], yn[1]) - np.exp(-1j * V * 1.0)) < 1e-13
    assert abs(yn[2] - (20.0 - 5.0 / 2000.0)) < 1e-13


def test_dp5_exit_and_accuracy():
    (s,), b = S.config1(n_traj=2, n_steps=1, jmax=3)
    o = oracle.OracleSystem(s)
    out = o.propagate(b, method="dp5", rtol=1e-10, atol=1e-10)
    assert np.all(out["status"] & oracle.STATUS["EXITED"])
    assert np.all(out["classical"][:, 0] >= b.R0) and np.all(out["classical"][:, 3] > 0)
    # same trajectories to the same end time with fine RK4
    for i in range(2):
        T = out["t_final"][i]
        ref = o.propagate(b.subset([i]), dt=[T / 40000], n_steps=[40000])
        assert np.max(np.abs(ref["P"][0] - out["P"][i])) < 1e-7
    fails = o.propagate(b, method="dp5", max_steps=10)
    assert np.all(fails["status"] & oracle.STATUS["MAX_STEPS"])
    under = o.propagate(b, method="dp5", rtol=1e-30, atol=1e-30, h_min=1e-3)
    assert np.all(under["status"] & oracle.STATUS["STEP_UNDERFLOW"])


def test_tables_at_a_run_of_knots_equal_the_whole_grid_spline():
    """The large-system oracle holds only the knots a trajectory touches, with the
    second derivatives of the whole grid's natural spline taken through the
    generator's rank-Q factors (the spline is linear in the data): they equal the
    oracle's own spline of every element, and so do the propagated results."""
    s = S.large_random_system(N=24, K=30, cfg_index=12, workers=0)
    full = oracle.OracleSystem(s)
    phi, v, H, scale = S.gp_rank_factors(s)
    ks = np.arange(22, 30)
    R_sub, M_sub, M2_sub = oracle.rank_q_knot_tables(s.R_grid, phi, v, H, ks, scale)
    assert np.array_equal(R_sub, s.R_grid[22:])
    assert np.max(np.abs(M_sub - s.M[22:])) <= 1e-15 * np.max(np.abs(s.M))
    M2 = full.M2.view(np.complex128).reshape(s.K, s.N, s.N)[22:]
    assert np.max(np.abs(M2_sub - M2)) <= 1e-12 * np.max(np.abs(M2))
    part = oracle.OracleSystem(s, knots=(R_sub, M_sub, M2_sub))
    rng = np.random.default_rng(5)
    b = S.mc_batch(s, 2, 1000.0, 6.0, [0, 3], rng, n_steps=60, dt=20.0)
    o1, o2 = full.propagate(b), part.propagate(b)
    assert np.all(o1["classical"][:, 0] > s.R_grid[22])        # stayed on the held knots
    assert np.max(np.abs(o1["P"] - o2["P"])) < 1e-12


def test_dual_number_derivative_matches_central_differences():
    (s,), b = S.config4(n_traj=2, n_steps=300, jmax=1)
    rng = np.random.default_rng(3)
    v = rng.standard_normal(s.theta.shape[0])
    dM = S.parametric_tables(s, v)
    o = oracle.OracleSystem(s, tangent_tables=dM)
    P, dP = o.tangent_rk4(b)
    h = 1e-5
    Pp = oracle.OracleSystem(s, tables=S.parametric_tables(s, s.theta + h * v)).propagate(b)["P"]
    Pm = oracle.OracleSystem(s, tables=S.parametric_tables(s, s.theta - h * v)).propagate(b)["P"]
    fd = (Pp - Pm) / (2 * h)
    assert np.max(np.abs(P - oracle.OracleSystem(s).propagate(b)["P"])) < 1e-13
    assert np.max(np.abs(dP - fd)) < 1e-6 * max(1.0, np.max(np.abs(fd)))
    assert np.max(np.abs(fd)) > 1e-4


# ------------------------------------------------------------------ cross sections, initial state

def test_cross_section_estimator_closed_form():
    """P = 1 inside b0 (midpoint sample of b on [0, b_max]) gives pi b0^2."""
    n, bmax, b0 = 20000, 20.0, 7.0
    bb = (np.arange(n) + 0.5) / n * bmax
    P = np.zeros((n, 2)); P[:, 1] = (bb < b0); P[:, 0] = 1 - P[:, 1]
    sig = oracle.cross_sections(np.zeros(n, np.int32), bb, P, np.array([0, 1], np.int32), 2, bmax)
    assert sig[0, 1] == pytest.approx(math.pi * b0 ** 2, rel=1e-6)
    assert sig[0, 0] + sig[0, 1] == pytest.approx(math.pi * bmax ** 2, rel=1e-9)


def test_lmax_relation_of_section_three():
    """Section III: b_max = 15 bohr at U = 12000 cm^-1 corresponds to l_max = 285 (H2O + H2)."""
    path = __file__.replace("test_oracle_pins.py", "golden/lmax_section3.txt")
    vals = dict(line.split("=") for line in open(path) if "=" in line and not line.startswith("#"))
    mu = U.amu_to_me(float(vals["mu_amu"]))
    E = U.cm_to_hartree(float(vals["U_cm"]))
    bmax = float(vals["b_max_bohr"])
    lmax = float(vals["l_max"])
    R = np.linspace(3.0, 30.0, 8)
    o = oracle.OracleSystem(make_system(R, [0.0], np.zeros((8, 1, 1)), mu=mu))
    out = o.propagate(init_channel=[0], E_coll=[E], b=[bmax], R0=[30.0], dt=[1.0], n_steps=[0])
    assert abs(out["classical"][0, 5] - lmax) < 0.5
