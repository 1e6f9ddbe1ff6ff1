"""GPU parity of decoupled (AT) dynamics (paper Section III: the quantum
equations propagated along a classical trajectory that does not feel the
quantum state, driven here by a tabulated potential U(R)).

* every schedule (per trajectory, binned and work list, RK4 and DP5) against
  the oracle's AT dynamics: 1e-9 with FP64 tables (DP5: 10 x rtol);
* many initial states on one trajectory: records that share (E_coll, b, R0)
  have bitwise identical classical results on the GPU, and the final
  amplitudes are linear in the initial ones;
* with an isotropic coupling M = V 1 the GPU's AT (U = V) and Ehrenfest runs
  agree, as the oracle's do;
* a batch asking for AT on a system without a driver fails cleanly.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S
from synth.systems import System

pytestmark = pytest.mark.gpu

RTOL = 1e-8


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.synchronize()
    c.close()


def driver_of(s):
    """The average diagonal of the tables: an isotropic driving potential."""
    return np.real(np.einsum("knn->k", s.M)) / s.N


def start(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)


@pytest.mark.parametrize("schedule", ["gemv", "binned", "queue"])
def test_at_rk4_matches_oracle(ctx, schedule):
    (s,), b = S.config1(n_traj=8, n_steps=500, jmax=3)
    U = driver_of(s)
    say("AT rk4 %s N=%d B=%d" % (schedule, s.N, b.B))
    sid = ctx.load_system(s)
    ctx.set_driver(sid, U)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule=schedule, dynamics="at", dt=b.dt,
                     n_steps=b.n_steps, **start(b))
    o = oracle.OracleSystem(s, driver=U).propagate(b)
    err = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    say("  max|dP| %.3e" % err)
    assert err < 1e-9
    assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < 1e-10
    assert np.max(np.abs(g["energy_err"] - o["energy_err"])) < 1e-10
    assert np.max(np.abs(g["angmom_err"])) == 0.0
    ctx.free_system(sid)


@pytest.mark.parametrize("schedule", ["queue", "binned"])
def test_at_dp5_matches_oracle(ctx, schedule):
    (s,), b = S.config1(n_traj=6, n_steps=1, jmax=3)
    U = driver_of(s)
    say("AT dp5 %s N=%d B=%d" % (schedule, s.N, b.B))
    sid = ctx.load_system(s)
    ctx.set_driver(sid, U)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, integrator="dp5", dynamics="at", rtol=RTOL,
                     atol=RTOL, max_steps=50000, h_min=1e-6, schedule=schedule, **start(b))
    o = oracle.OracleSystem(s, driver=U).propagate(b, method="dp5", rtol=RTOL, atol=RTOL,
                                                   max_steps=50000, h_min=1e-6)
    assert np.all(g["status"] & 1) and np.max(np.abs(g["steps"] - o["steps"])) <= 2
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 10 * RTOL
    ctx.free_system(sid)


@pytest.mark.parametrize("schedule", ["gemv", "binned"])
def test_at_many_initial_states_share_one_path(ctx, schedule):
    """Four trajectories x all N initial states in one batch (the AT workload):
    shared classical results, and amplitudes linear in the initial ones."""
    (s,), b0 = S.config1(n_traj=4, n_steps=300, jmax=2)
    U = driver_of(s)
    N = s.N
    idx = np.repeat(np.arange(b0.B), N)
    b = b0.subset(idx)
    b.init_channel = np.tile(np.arange(N, dtype=np.int32), b0.B)
    say("AT shared paths %s N=%d, %d x %d" % (schedule, N, b0.B, N))
    sid = ctx.load_system(s)
    ctx.set_driver(sid, U)
    common = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                  n_steps=b.n_steps)
    g = ctx.run_host([sid] * b.B, [N] * b.B, schedule=schedule, dynamics="at", **common)
    cl = g["classical"].reshape(b0.B, N, 6)
    assert np.all(cl == cl[:, :1, :])
    A = g["a_final"].reshape(b0.B, N, N)          # A[traj, initial, final]
    # a superposition of two initial states propagates to the same superposition
    al, be = 0.6, 0.8j
    a0 = np.zeros((b0.B, N), complex)
    a0[:, 1] = al
    a0[:, 3] = be
    sup = ctx.run_host([sid] * b0.B, [N] * b0.B, schedule=schedule, dynamics="at", a0=a0,
                       E_coll=b0.E_coll, b=b0.b, R0=b0.R0, dt=b0.dt, n_steps=b0.n_steps)
    lin = al * A[:, 1, :] + be * A[:, 3, :]
    assert np.max(np.abs(sup["a_final"].reshape(b0.B, N) - lin)) < 1e-12
    ctx.free_system(sid)


def test_at_equals_ehrenfest_for_isotropic_coupling_on_gpu(ctx):
    (s,), b = S.config1(n_traj=6, n_steps=6000, jmax=3)
    U = driver_of(s)
    M = np.zeros_like(s.M)
    for n in range(s.N):
        M[:, n, n] = U
    iso = System("iso", s.R_grid, s.E, M, s.jx_row, s.jx_col, s.jx_val, s.mu,
                 s.level_of_channel, s.n_levels)
    say("AT vs Ehrenfest, isotropic coupling N=%d" % s.N)
    sid = ctx.load_system(iso)
    ctx.set_driver(sid, U)
    common = dict(dt=b.dt, n_steps=b.n_steps, schedule="gemv", **start(b))
    eh = ctx.run_host([sid] * b.B, [s.N] * b.B, **common)
    at = ctx.run_host([sid] * b.B, [s.N] * b.B, dynamics="at", **common)
    assert np.max(np.abs(eh["P"] - at["P"])) < 1e-9
    ctx.free_system(sid)


def test_at_without_driver_is_rejected(ctx, gpu_lib):
    (s,), b = S.config1(n_traj=2, n_steps=5, jmax=1)
    sid = ctx.load_system(s)
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.run_host([sid] * b.B, [s.N] * b.B, dynamics="at", dt=b.dt, n_steps=b.n_steps,
                     **start(b))
    assert e.value.code == gpu_lib.ERR_STATE
    ctx.free_system(sid)
