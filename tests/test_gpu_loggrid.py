"""Propagation on the paper's radial grid: 63 points spaced logarithmically from
3 to 30 bohr (Section III), so knot spacings differ by a factor of ten across the
grid.  The interval is then found by binary search and the spline weights use
unequal spacings -- the branch uniform grids skip.  Every schedule, both
integrators, FP64 and FP32 tables, real and complex couplings, against the oracle:
FP64 fixed-step RK4 within 1e-9, adaptive DP5 within 10 rtol with the oracle's
step counts, FP32 tables within 1e-4 -- per channel.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import coupling as CP
from synth import systems as S, units as U

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


def grid_ang():
    return U.bohr_to_ang(CP.log_grid(63, 3.0, 30.0))


def rotor_on_log_grid():
    s = S.rotor_atom_system(jmax=3, R_ang=grid_ang())
    assert s.K == 63 and abs(s.R_grid[0] - 3.0) < 1e-12 and abs(s.R_grid[-1] - 30.0) < 1e-12
    h = np.diff(s.R_grid)
    assert h.max() / h.min() > 9.0
    return s


def batch_for(s, n_traj=6, n_steps=800, seed=31):
    rng = np.random.default_rng(seed)
    init = np.arange(min(4, s.N))
    return S.mc_batch(s, n_traj, rng.uniform(300.0, 900.0, n_traj), 5.0, init, rng,
                      n_steps=n_steps)


def start(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)


def turning_points(g):
    """Smallest R reached (the classical state is at the end; the run covers the
    inner grid if the trajectories came back out)."""
    return g["classical"].reshape(-1, 6)[:, 0]


@pytest.mark.parametrize("storage", ["R64", "R32"])
@pytest.mark.parametrize("schedule", ["gemv", "binned", "queue"])
def test_rk4_on_log_grid(ctx, schedule, storage):
    s = rotor_on_log_grid()
    b = batch_for(s)
    say("log grid RK4 %s %s N=%d B=%d" % (schedule, storage, s.N, b.B))
    sid = ctx.load_system(s, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, dt=b.dt, n_steps=b.n_steps, schedule=schedule,
                     **start(b))
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b)
    assert np.all(g["status"] == o["status"])
    # the trajectories went in and came out again: both ends of the grid were used
    assert np.all(g["classical"].reshape(-1, 6)[:, 3] > 0)
    d = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    say("  max|dP| = %.3e" % d)
    assert d < (1e-9 if storage == "R64" else 1e-4)
    dc = np.max(np.abs(g["classical"].reshape(b.B, 6) - o["classical"]) / (1 + np.abs(o["classical"])))
    assert dc < (1e-9 if storage == "R64" else 1e-5)


@pytest.mark.parametrize("schedule", ["queue", "binned"])
def test_dp5_on_log_grid(ctx, schedule):
    s = rotor_on_log_grid()
    b = batch_for(s, n_traj=5, n_steps=1)
    say("log grid DP5 %s N=%d B=%d" % (schedule, s.N, b.B))
    sid = ctx.load_system(s, storage="R64")
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, integrator="dp5", rtol=RTOL, atol=RTOL,
                     max_steps=50000, h_min=1e-6, schedule=schedule, **start(b))
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                                         h_min=1e-6)
    say("  steps gpu %s oracle %s" % (g["steps"].tolist(), o["steps"].tolist()))
    assert np.all(g["status"] & 1) and np.all(o["status"] & 1)
    assert np.array_equal(g["steps"], o["steps"]) and np.array_equal(g["rejects"], o["rejects"])
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 10 * RTOL
    # the step sizes follow the error estimates, which differ in rounding: end
    # times agree to the accumulated rounding of the step sequence
    assert np.max(np.abs(g["t_final"] - o["t_final"]) / o["t_final"]) < 1e-7


@pytest.mark.parametrize("storage", ["C128", "C64"])
@pytest.mark.parametrize("schedule", ["gemv", "binned"])
def test_complex_tables_on_log_grid(ctx, schedule, storage):
    s = S.large_random_system(N=40, cfg_index=9, R_ang=grid_ang(), workers=0)
    b = batch_for(s, n_traj=4, n_steps=700, seed=32)
    say("log grid complex %s %s N=%d" % (schedule, storage, s.N))
    sid = ctx.load_system(s, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, dt=b.dt, n_steps=b.n_steps, schedule=schedule,
                     **start(b))
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b)
    d = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    say("  max|dP| = %.3e" % d)
    assert d < (1e-9 if storage == "C128" else 1e-4)
