"""GPU parity of adaptive Dormand-Prince 5(4) on the binned schedule.

Every unfinished trajectory makes one attempt per round, each of its six stage
evaluations a knot-binned product on the matrix cores.  Tableau, error norm,
controller and stopping rules are the work-list schedule's; the right-hand sides
differ from the oracle's and the work-list schedule's only in summation order,
so the accept/reject decisions agree except when an error estimate lands within
rounding of 1: step counts may differ by a few steps and final probabilities
are compared at 10 x rtol (FP64 tables) and 1e-4 (FP32 tables), as for the
work-list schedule.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S

pytestmark = pytest.mark.gpu

RTOL = 1e-8
DP5 = dict(integrator="dp5", rtol=RTOL, atol=RTOL, max_steps=50000, h_min=1e-6)


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.synchronize()
    c.close()


def start(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)


def test_binned_dp5_fp64_matches_oracle_and_work_list(ctx):
    s = S.rotor_atom_system(jmax=5)
    rng = np.random.default_rng(20231203)
    init = np.where(s.labels["j"] == 2)[0]
    b = S.mc_batch(s, 12, 500.0, 10.0, init, rng, n_steps=1)
    say("binned dp5 rotor N=%d R64 B=%d" % (s.N, b.B))
    sid = ctx.load_system(s)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="binned", **start(b), **DP5)
    q = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", **start(b), **DP5)
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                                         h_min=1e-6)
    say("  steps binned %s work-list %s oracle %s" % (g["steps"].tolist(), q["steps"].tolist(),
                                                      o["steps"].tolist()))
    assert np.all(g["status"] & 1) and np.all(o["status"] & 1)            # exited
    assert np.max(np.abs(g["steps"] - o["steps"])) <= 2
    assert np.max(np.abs(g["steps"] - q["steps"])) <= 2
    P = g["P"].reshape(b.B, s.N)
    assert np.max(np.abs(P - o["P"])) < 10 * RTOL
    assert np.max(np.abs(P - q["P"].reshape(b.B, s.N))) < 10 * RTOL
    assert np.max(np.abs(g["t_final"] - o["t_final"]) / o["t_final"]) < 1e-3
    assert np.max(np.abs(g["energy_err"] - o["energy_err"])) < 1e-8
    assert np.max(np.abs(g["norm_err"] - o["norm_err"])) < 1e-8


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_binned_dp5_complex_tables(ctx, storage):
    (s,), b = S.config2(n_traj=6, jmax=3)
    say("binned dp5 config2 reduced N=%d %s B=%d" % (s.N, storage, b.B))
    sid = ctx.load_system(s, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="binned", **start(b), **DP5)
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                                         h_min=1e-6)
    d = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    say("  steps binned %s oracle %s, max|dP| %.2e" % (g["steps"].tolist(), o["steps"].tolist(), d))
    assert np.array_equal(g["status"] & 1, o["status"] & 1)
    assert d < (10 * RTOL if storage == "C128" else 1e-4)
    if storage == "C128":
        assert np.max(np.abs(g["steps"] - o["steps"])) <= 2


def test_binned_dp5_stopping_rules(ctx):
    """A step limit and a step floor stop trajectories with the work-list
    schedule's status bits and counts."""
    s = S.rotor_atom_system(jmax=3)
    rng = np.random.default_rng(7)
    b = S.mc_batch(s, 5, 500.0, 8.0, np.arange(4), rng, n_steps=1)
    sid = ctx.load_system(s)
    for kw in (dict(DP5, max_steps=10), dict(DP5, rtol=1e-30, atol=1e-30, h_min=1e-3)):
        g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="binned", **start(b), **kw)
        q = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", **start(b), **kw)
        say("  limits %s: status binned %s work-list %s, steps %s %s" % (
            {k: kw[k] for k in ("max_steps", "h_min", "rtol")}, g["status"].tolist(),
            q["status"].tolist(), g["steps"].tolist(), q["steps"].tolist()))
        assert np.array_equal(g["status"], q["status"])
        assert np.array_equal(g["steps"], q["steps"])
        assert np.max(np.abs(g["rejects"] - q["rejects"])) <= 1
    ctx.free_system(sid)


def test_binned_dp5_restart_from_a_given_state(ctx):
    """A run stopped at 15 accepted steps and continued from its amplitudes,
    classical state and time (a0, classical0, t0) ends where the work-list
    schedule's chain of the same two calls ends."""
    s = S.rotor_atom_system(jmax=4)
    rng = np.random.default_rng(99)
    init = np.where(s.labels["j"] == 2)[0]
    b = S.mc_batch(s, 6, 400.0, 9.0, init, rng, n_steps=1)
    sid = ctx.load_system(s)
    ends = {}
    for sched in ("binned", "queue"):
        g1 = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule=sched, **start(b),
                          **dict(DP5, max_steps=15))
        assert np.all(g1["status"] & 2)                       # stopped at the step limit
        g2 = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule=sched, a0=g1["a_final"],
                          classical0=g1["classical"], t0=g1["t_final"], **DP5)
        ends[sched] = g2
    ctx.free_system(sid)
    say("  restart: steps binned %s work-list %s" % (ends["binned"]["steps"].tolist(),
                                                     ends["queue"]["steps"].tolist()))
    assert np.array_equal(ends["binned"]["status"], ends["queue"]["status"])
    assert np.max(np.abs(ends["binned"]["steps"] - ends["queue"]["steps"])) <= 2
    assert np.max(np.abs(ends["binned"]["P"] - ends["queue"]["P"])) < 10 * RTOL


def test_default_schedule_splits_an_adaptive_batch(ctx):
    """One call, default schedule: the trajectories of a large dense system that
    holds many of them run on the binned schedule (a second stream), the rest on
    the work list, concurrently.  Each share equals the same trajectories run on
    their schedule alone: bit for bit on the binned share (its products do not
    depend on which other trajectories share a knot), to rounding on the work
    list (whose shape the autotuner may choose differently in each call)."""
    big = S.large_random_system(N=512, K=60, cfg_index=11, workers=0)
    rng = np.random.default_rng(41)
    bb = S.mc_batch(big, 256, rng.uniform(800.0, 1500.0, 256), 8.0, np.arange(8), rng, n_steps=1)
    small = S.rotor_atom_system(jmax=3)
    init = np.where(small.labels["j"] == 2)[0]
    bs = S.mc_batch(small, 9, 500.0, 10.0, init, rng, n_steps=1)
    say("split adaptive batch: N=%d x %d (binned share) + N=%d x %d (work list)" % (
        big.N, bb.B, small.N, bs.B))
    s1 = ctx.load_system(big, storage="C64")
    s2 = ctx.load_system(small, storage="R64")
    order = rng.permutation(bb.B + bs.B)
    cat = lambda x, y: np.concatenate([np.asarray(x), np.asarray(y)])[order]
    ids = cat(np.full(bb.B, s1), np.full(bs.B, s2))
    Ns = cat(np.full(bb.B, big.N), np.full(bs.B, small.N))
    kw = dict(init_channel=cat(bb.init_channel, bs.init_channel), E_coll=cat(bb.E_coll, bs.E_coll),
              b=cat(bb.b, bs.b), R0=cat(bb.R0, bs.R0))
    g = ctx.run_host(ids, Ns, **kw, **DP5)
    gb = ctx.run_host([s1] * bb.B, [big.N] * bb.B, schedule="binned", **start(bb), **DP5)
    gq = ctx.run_host([s2] * bs.B, [small.N] * bs.B, schedule="queue", **start(bs), **DP5)
    ctx.free_system(s1)
    ctx.free_system(s2)
    offs = np.concatenate([[0], np.cumsum(Ns)])
    inv = np.argsort(order)
    for i in range(bb.B):
        pos = inv[i]
        assert np.array_equal(g["P"][offs[pos]:offs[pos + 1]], gb["P"][i * big.N:(i + 1) * big.N])
        assert g["steps"][pos] == gb["steps"][i] and g["t_final"][pos] == gb["t_final"][i]
    for i in range(bs.B):
        pos = inv[bb.B + i]
        assert np.max(np.abs(g["P"][offs[pos]:offs[pos + 1]] -
                             gq["P"][i * small.N:(i + 1) * small.N])) < 1e-12
    assert np.all(g["status"] & 1)
    say("  steps %d..%d, all exited" % (g["steps"].min(), g["steps"].max()))
