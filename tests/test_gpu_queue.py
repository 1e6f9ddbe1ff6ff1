"""GPU parity of the work-list schedule (one step attempt per launch for every
unfinished trajectory, several once few are left, finished ones retired between
chunks, chunks replayed as HIP graphs).

* Fixed-step RK4 on a ragged batch computes exactly the arithmetic of the
  per-trajectory kernel when both use the same workgroup shape: the results are
  compared bit for bit, with graphs on and off, for several chunk sizes and for
  one or several attempts per launch.
* Adaptive Dormand-Prince 5(4) against the FP64 oracle's DP5 (same tableau,
  error norm and controller): the two take the same accept/reject decisions
  except when an error estimate lands within rounding of 1, so step counts may
  differ by a few steps and final probabilities are compared at 10 x rtol (FP64
  tables) and 1e-4 (FP32 tables).
* Uneven batches mixing systems of different size and kind in one call.
* The autotuner's choice is reported and the tuned run still meets the bar.
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


def rotor_batch(jmax, n, seed, n_steps=1, U_cm=500.0, b_max=10.0):
    s = S.rotor_atom_system(jmax=jmax)
    rng = np.random.default_rng(seed)
    init = np.where(s.labels["j"] == min(2, jmax))[0]
    return s, S.mc_batch(s, n, U_cm, b_max, init, rng, n_steps=n_steps)


def start(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)


def same(g1, g2):
    for k in ("a_final", "classical", "t_final", "steps", "rejects", "status", "energy_err",
              "norm_err", "angmom_err"):
        assert np.array_equal(g1[k], g2[k]), k


def test_queue_rk4_ragged_bitwise_equals_per_trajectory(ctx):
    """Step counts 0, 1, ... 257 in one batch; shape fixed (autotuner off)."""
    s, b = rotor_batch(4, 24, 11, n_steps=257)
    b.n_steps = np.array([0, 1, 2, 3, 5, 8, 13, 21, 34, 55, 89, 144, 233, 257, 200, 150, 100,
                          50, 25, 12, 6, 3, 2, 257], np.int64)
    say("queue rk4 ragged N=%d B=%d" % (s.N, b.B))
    sid = ctx.load_system(s)
    ctx.set_option("autotune", 0)
    try:
        common = dict(start(b), dt=b.dt, n_steps=b.n_steps)
        ref = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="gemv", **common)
        # per_launch: steps per launch once few trajectories are left (here from the start)
        for graphs, chunk, per in ((1, 16, 4), (0, 16, 4), (1, 1, 4), (1, 7, 4), (1, 16, 1),
                                   (0, 5, 1), (1, 3, 64), (0, 16, 7)):
            say("  graphs=%d chunk=%d per_launch=%d" % (graphs, chunk, per))
            ctx.set_option("graphs", graphs)
            ctx.set_option("chunk", chunk)
            ctx.set_option("per_launch", per)
            g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", **common)
            same(ref, g)
        assert np.array_equal(ref["steps"], b.n_steps)
    finally:
        ctx.set_option("graphs", 1)
        ctx.set_option("chunk", 16)
        ctx.set_option("per_launch", 1)
        ctx.set_option("autotune", 1)
    ctx.free_system(sid)


def test_queue_rk4_matches_oracle(ctx):
    s, b = rotor_batch(3, 12, 5, n_steps=400)
    say("queue rk4 vs oracle N=%d B=%d" % (s.N, b.B))
    sid = ctx.load_system(s)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", dt=b.dt, n_steps=b.n_steps,
                     **start(b))
    o = oracle.OracleSystem(s).propagate(b)
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 1e-9
    ctx.free_system(sid)


def test_dp5_fp64_matches_oracle(ctx):
    s, b = rotor_batch(5, 10, 20231202)
    say("dp5 rotor N=%d R64 B=%d" % (s.N, b.B))
    sid = ctx.load_system(s)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, **start(b), **DP5)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                                         h_min=1e-6)
    say("  steps gpu %s oracle %s" % (g["steps"].tolist(), o["steps"].tolist()))
    assert np.all(g["status"] & 1) and np.all(o["status"] & 1)           # exited
    assert np.max(np.abs(g["steps"] - o["steps"])) <= 2
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 10 * RTOL
    assert np.max(np.abs(g["t_final"] - o["t_final"]) / o["t_final"]) < 1e-3
    # the adaptive scheme's own conservation errors (about 1e-5 in energy at
    # these step counts) are the oracle's: same discrete map, same defects
    assert np.max(np.abs(g["energy_err"] - o["energy_err"])) < 1e-8
    assert np.max(np.abs(g["norm_err"] - o["norm_err"])) < 1e-8
    ctx.free_system(sid)


def mixed(n_each, jmax):
    systems, b = S.config3(n_traj=sum(n_each), split=tuple(np.array(n_each) / sum(n_each)),
                           jmax=jmax)
    return systems, b


@pytest.mark.parametrize("fam", ["fp64", "fp32"])
def test_dp5_uneven_mixed_batch(ctx, fam):
    """Three systems (rotor, rotor-rotor, asymmetric top) of different N and kind,
    log-uniform collision energies, shuffled, in one call."""
    systems, b = mixed((7, 5, 3), (4, 1, 2))
    kinds = ["R64", "R64", "C128"] if fam == "fp64" else ["R32", "R32", "C64"]
    say("dp5 uneven mix %s N=%s B=%d" % (fam, [x.N for x in systems], b.B))
    ids = [ctx.load_system(x, storage=k) for x, k in zip(systems, kinds)]
    sids = np.array([ids[i] for i in b.system_index])
    Ns = np.array([systems[i].N for i in b.system_index])
    g = ctx.run_host(sids, Ns, **start(b), **DP5)
    offs = np.concatenate([[0], np.cumsum(Ns)])
    # FP64: the same accepted steps as the oracle, so every channel agrees to the
    # tolerance.  FP32: the step sequence may differ from the oracle's by a step or
    # two, and the exit time with it; every channel is compared with the exact
    # solution at the GPU trajectory's own end time (the oracle's RK4 from the
    # start to that time in steps a hundred times finer than the adaptive ones).
    tol = 10 * RTOL if fam == "fp64" else 1e-4
    worst = 0.0
    for si, x in enumerate(systems):
        idx = np.where(b.system_index == si)[0]
        ox = oracle.OracleSystem(x)
        o = ox.propagate(b.subset(idx), method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                         h_min=1e-6)
        if fam == "fp32":
            sub = b.subset(idx)
            n_fine = np.maximum(2000, 100 * g["steps"][idx]).astype(np.int64)
            ref = ox.propagate(sub, dt=g["t_final"][idx] / n_fine, n_steps=n_fine)["P"]
        for k, i in enumerate(idx):
            dP = g["P"][offs[i]:offs[i + 1]] - (o["P"][k] if fam == "fp64" else ref[k])
            worst = max(worst, np.max(np.abs(dP)))
            assert g["status"][i] & 1
            assert abs(int(g["steps"][i]) - int(o["steps"][k])) <= 3 + 0.01 * o["steps"][k]
    say("  max|dP| = %.3e, steps %d..%d" % (worst, g["steps"].min(), g["steps"].max()))
    assert worst < tol
    # the same batch with graphs off, another chunk size and one or seven attempts
    # per launch: identical results
    for per in (4, 7):
        ctx.set_option("graphs", 0)
        ctx.set_option("chunk", 5)
        ctx.set_option("per_launch", per)
        try:
            g2 = ctx.run_host(sids, Ns, **start(b), **DP5)
        finally:
            ctx.set_option("graphs", 1)
            ctx.set_option("chunk", 16)
            ctx.set_option("per_launch", 1)
        same(g, g2)
    for i in ids:
        ctx.free_system(i)


def test_dp5_failure_statuses(ctx):
    s, b = rotor_batch(2, 3, 99)
    say("dp5 failure statuses N=%d" % s.N)
    sid = ctx.load_system(s)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, **start(b), **dict(DP5, max_steps=10))
    assert np.all(g["status"] & 2) and np.all(g["steps"] == 10)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=10,
                                         h_min=1e-6)
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 10 * RTOL
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, **start(b),
                     **dict(DP5, rtol=1e-30, atol=1e-30, h_min=1e-3))
    assert np.all(g["status"] & 4)
    ctx.free_system(sid)


def test_autotuner_reports_and_meets_the_bar(ctx):
    """N = 256 rotor-rotor system in FP32 tables: two candidate shapes (64 threads
    x 4 rows, 128 threads x 2 rows); the tuned run matches the oracle."""
    (s,), b = S.config4(n_traj=48, n_steps=60)
    say("autotune N=%d R32 B=%d" % (s.N, b.B))
    sid = ctx.load_system(s, storage="R32")
    ctx.set_option("reset_tuning")
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", dt=b.dt, n_steps=b.n_steps,
                     **start(b))
    rep = [e for e in ctx.tuning_report() if e["npad"] == 256 and e["dtype"] == 2]
    say("  report %s" % rep)
    assert len(rep) == 1 and rep[0]["tuned"] and len(rep[0]["candidates"]) == 2
    assert all(c["ms"] > 0 for c in rep[0]["candidates"])
    o = oracle.OracleSystem(s).propagate(b)
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"])) < 1e-4
    # the decision is kept: a second run reuses it and reproduces the first exactly
    g2 = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", dt=b.dt, n_steps=b.n_steps,
                      **start(b))
    same(g, g2)
    ctx.free_system(sid)


@pytest.mark.parametrize("storage", ["R64", "R32"])
def test_split_row_form_matches_oracle(ctx, storage):
    """The split-row form (8 waves that each hold all rows and stream an eighth of
    the stored rows, partial sums added in LDS) forced for a whole batch: RK4 and
    DP5 against the oracle, and RK4 against the row-split form."""
    (s,), b = S.config4(n_traj=6, n_steps=80)
    say("split-row form N=%d %s" % (s.N, storage))
    sid = ctx.load_system(s, storage=storage)
    common = dict(start(b), dt=b.dt, n_steps=b.n_steps)
    tol = 1e-9 if storage == "R64" else 1e-4
    ctx.set_option("tail", 2)
    try:
        g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="queue", **common)
        d = ctx.run_host([sid] * b.B, [s.N] * b.B, **start(b), **DP5)
    finally:
        ctx.set_option("tail", 1)
    ref = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="gemv", **common)
    o = oracle.OracleSystem(s).propagate(b)
    od = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=RTOL, atol=RTOL, max_steps=50000,
                                          h_min=1e-6)
    e_rk = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    e_dp = np.max(np.abs(d["P"].reshape(b.B, s.N) - od["P"]))
    say("  rk4 |dP| %.3e  dp5 |dP| %.3e  vs row-split %.3e" % (
        e_rk, e_dp, np.max(np.abs(g["P"] - ref["P"]))))
    assert e_rk < tol
    assert e_dp < (10 * RTOL if storage == "R64" else 1e-4)
    assert np.max(np.abs(g["P"] - ref["P"])) < tol
    assert np.all(d["status"] & 1) and np.max(np.abs(d["steps"] - od["steps"])) <= 3
    ctx.free_system(sid)
