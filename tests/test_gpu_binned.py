"""GPU parity of the R-binned lockstep schedule (matrix-core products per knot).

Same bars as the per-trajectory kernels: FP64 tables within 1e-9 of the oracle,
FP32 tables within 1e-4.  At the full N = 969 size of the benchmark the binned
and per-trajectory schedules are compared on the whole 4096-trajectory batch
and the oracle checks a sample of trajectories.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    yield c
    c.synchronize()
    c.close()


def run(ctx, sid, s, b, schedule, **kw):
    args = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                n_steps=b.n_steps, schedule=schedule)
    args.update(kw)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, **args)
    g["P"] = g["P"].reshape(b.B, s.N)
    g["a_final"] = g["a_final"].reshape(b.B, s.N)
    return g


def test_binned_config1_fp64(ctx):
    (s,), b = S.config1()
    say("binned config1 N=49 B=64 2000 steps R64")
    sid = ctx.load_system(s)
    g = run(ctx, sid, s, b, "binned")
    o = oracle.OracleSystem(s).propagate(b)
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < 1e-9
    assert np.max(np.abs(g["energy_err"] - o["energy_err"])) < 1e-9
    assert np.max(np.abs(g["angmom_err"] - o["angmom_err"])) < 1e-9
    assert np.array_equal(g["steps"], b.n_steps) and np.all(g["status"] == 0)
    ctx.free_system(sid)


def test_binned_config2_reduced(ctx):
    (s,), b = S.config2(n_traj=6, jmax=3)
    b.n_steps[:] = np.minimum(b.n_steps, 2500)
    say("binned config2 reduced N=84 C128 and C64")
    o = oracle.OracleSystem(s).propagate(b)
    sid = ctx.load_system(s, storage="C128")
    g = run(ctx, sid, s, b, "binned")
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    ctx.free_system(sid)
    sid = ctx.load_system(s, storage="C64")
    g = run(ctx, sid, s, b, "binned")
    err = np.max(np.abs(g["P"] - o["P"]))
    say("binned config2 reduced fp32 max|dP| = %.3e" % err)
    assert err < 1e-4
    ctx.free_system(sid)


def test_binned_config4_and_ragged_steps(ctx):
    (s,), b = S.config4(n_traj=5, n_steps=500)
    b.n_steps[:] = [500, 120, 0, 333, 499]
    say("binned config4 N=256 R64 ragged steps")
    o = oracle.OracleSystem(s).propagate(b)
    sid = ctx.load_system(s)
    g = run(ctx, sid, s, b, "binned")
    assert np.array_equal(g["steps"], b.n_steps)
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    assert np.max(np.abs(g["t_final"] - o["t_final"])) < 1e-9 * np.max(o["t_final"])
    ctx.free_system(sid)


@pytest.fixture(scope="module")
def full_size():
    return S.config2(n_traj=4096, full_collision=False, window_steps=2)


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_binned_full_size_bench_population(ctx, full_size, storage):
    """N = 969, 4096 mid-collision trajectories (the benchmark's launch), 2 RK4 steps."""
    (s,), b = full_size
    say("full-size N=969 B=4096 %s: binned vs per-trajectory" % storage)
    sid = ctx.load_system(s, storage=storage)
    gb = run(ctx, sid, s, b, "binned")
    gg = run(ctx, sid, s, b, "gemv")
    d = np.max(np.abs(gb["P"] - gg["P"]))
    say("full-size %s max|P_binned - P_gemv| = %.3e" % (storage, d))
    assert d < (1e-12 if storage == "C128" else 1e-5)
    ctx.free_system(sid)
    sample = [0, 1, 2047, 4095]
    o = oracle.OracleSystem(s).propagate(b.subset(sample))
    tol = 1e-9 if storage == "C128" else 1e-4
    assert np.max(np.abs(gb["P"][sample] - o["P"])) < tol
    assert np.max(np.abs(gg["P"][sample] - o["P"])) < tol


def test_profiled_table_bytes(ctx):
    """The algorithmic table bytes reported with the kernel timings.

    Per-trajectory RK4: (4 n_steps + 1) right-hand sides x 4 slices of N x Npad
    elements.  Binned: trajectories that stay inside one spline interval occupy
    exactly its two knots at every stage, each read as a value and a
    second-derivative slice: (4 n_steps + 1) stages x 2 knots x 2 slices."""
    (s,), b = S.config1(n_traj=6, n_steps=3, jmax=3)      # N = 16, real FP64 tables
    b.R0[:] = 0.5 * (s.R_grid[100] + s.R_grid[101])      # mid-interval, far from both knots
    b.dt[:] = 1.0                                         # moves ~1e-3 bohr in 3 steps
    say("profiled table bytes N=%d" % s.N)
    sid = ctx.load_system(s, storage="R64")
    npad = 16
    per_slice = s.N * npad * 8
    for sched, expect in (("gemv", b.B * (4 * 3 + 1) * 4 * per_slice),
                          ("binned", (4 * 3 + 1) * 2 * 2 * per_slice)):
        ctx.set_profiling(True)
        run(ctx, sid, s, b, sched)
        ms, n, by = ctx.profile_read(with_bytes=True)
        ctx.set_profiling(False)
        say("  %s: %d launches, %.0f bytes (expected %d)" % (sched, n, by, expect))
        assert n > 0 and by == expect
    ctx.free_system(sid)


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_binned_wide_system_c_outside_lds(ctx, storage):
    """N = 2100 (padded past 2048 columns): the combine keeps c in device memory
    instead of LDS.  Channels come in degenerate pairs (2i, 2i+1) coupled by a
    real-symmetric J_x, so every row's Coriolis term reads c of another row.
    Binned against the per-trajectory schedule and against the oracle (FP64
    tables 1e-12 / 1e-9, FP32 tables 1e-4)."""
    s = S.large_random_system(N=2100, K=12, cfg_index=7)
    s.E = np.repeat(s.E[0::2], 2)
    s.level_of_channel = (np.arange(s.N) // 2).astype(np.int32)
    s.n_levels = s.N // 2
    n = np.arange(0, s.N, 2, dtype=np.int32)
    s.jx_row = np.concatenate([n, n + 1])
    s.jx_col = np.concatenate([n + 1, n])
    s.jx_val = np.tile(0.5 + 0.25 * np.cos(n), 2)
    rng = np.random.default_rng(21)
    b = S.mc_batch(s, 3, 600.0, 6.0, [0, 1000, 2099], rng, n_steps=12, dt=20.0,
                   R0_bohr=0.5 * (s.R_grid[6] + s.R_grid[7]))
    say("binned N=%d %s (c outside LDS), %d trajectories x %d steps" % (s.N, storage, b.B, 12))
    sid = ctx.load_system(s, storage=storage)
    gb = run(ctx, sid, s, b, "binned")
    gg = run(ctx, sid, s, b, "gemv")
    ctx.free_system(sid)
    fp64 = storage == "C128"
    d = np.max(np.abs(gb["P"] - gg["P"]))
    say("  max|P_binned - P_gemv| = %.3e" % d)
    assert d < (1e-12 if fp64 else 1e-5)
    assert np.max(np.abs(gb["classical"] - gg["classical"]) / (1 + np.abs(gg["classical"]))) < \
        (1e-12 if fp64 else 1e-6)
    o = oracle.OracleSystem(s).propagate(b.subset([1]))
    d = np.max(np.abs(gb["P"][1] - o["P"][0]))
    say("  max|P_binned - P_oracle| = %.3e" % d)
    assert d < (1e-9 if fp64 else 1e-4)


@pytest.fixture(scope="module")
def n4096():
    """N = 4096 random Hermitian tables on 12 knots (the large workload's size; the
    grid is short so the oracle can hold it), two trajectories in the middle."""
    s = S.large_random_system(N=4096, K=12, cfg_index=8)
    rng = np.random.default_rng(22)
    b = S.mc_batch(s, 2, 1000.0, 4.0, [0, 7], rng, n_steps=10, dt=20.0,
                   R0_bohr=0.5 * (s.R_grid[6] + s.R_grid[7]))
    return s, b


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_binned_n4096_rk4_against_oracle(ctx, n4096, storage):
    """The shape of every stage of the large workload: 4096 channels, the c columns
    and phases outside LDS, the FP32 product summing all 8192 reals of a row in the
    matrix-core accumulators."""
    s, b = n4096
    say("binned N=4096 %s RK4: %d trajectories x %d steps" % (storage, b.B, b.n_steps[0]))
    sid = ctx.load_system(s, storage=storage)
    g = run(ctx, sid, s, b, "binned")
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b)
    d = np.max(np.abs(g["P"] - o["P"]))
    say("  max|dP| = %.3e (norm err %.2e)" % (d, np.max(np.abs(g["norm_err"]))))
    assert d < (1e-9 if storage == "C128" else 1e-4)
    assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < \
        (1e-9 if storage == "C128" else 1e-6)


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_binned_n4096_dp5_against_oracle(ctx, n4096, storage):
    """Adaptive steps at N = 4096 (the binned DP5 stage kernels with c outside
    LDS): the starting step and four accepted steps against the oracle's."""
    s, b = n4096
    say("binned N=4096 %s DP5, 4 accepted steps" % storage)
    sid = ctx.load_system(s, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                     b=b.b, R0=b.R0, integrator="dp5", rtol=1e-8, atol=1e-8, max_steps=4,
                     h_min=1e-6, schedule="binned")
    ctx.free_system(sid)
    o = oracle.OracleSystem(s).propagate(b, method="dp5", rtol=1e-8, atol=1e-8, max_steps=4,
                                         h_min=1e-6)
    assert np.all(g["steps"] == 4) and np.all(o["steps"] == 4)
    if storage == "C128":
        assert np.array_equal(g["rejects"], o["rejects"])
        assert np.max(np.abs(g["t_final"] - o["t_final"]) / o["t_final"]) < 1e-9
    d = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
    say("  max|dP| = %.3e, t %s vs %s" % (d, g["t_final"], o["t_final"]))
    assert d < (1e-7 if storage == "C128" else 1e-4)


@pytest.mark.parametrize("schedule", ["binned", "gemv", "queue"])
def test_trajectory_that_overflows_stops_alone(ctx, schedule):
    """Initial amplitudes of 1e200 in one trajectory overflow its norm and force in the
    first step: it stops after that step with the non-finite status bit, while the
    others (sharing its bins, on the binned schedule) run on as they do without it:
    bit for bit on the binned and per-trajectory schedules; on the work-list
    schedule, whose workgroup shape may change with the batch, to rounding."""
    (s,), b = S.config1(n_traj=4, n_steps=40)
    say("%s: one overflowing trajectory among 4 (N=%d)" % (schedule, s.N))
    sid = ctx.load_system(s)
    a0 = np.zeros((b.B, s.N), np.complex128)
    a0[np.arange(b.B), b.init_channel] = 1.0
    a0[2, b.init_channel[2]] = 1e200
    kw = dict(E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps, schedule=schedule)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, a0=a0.reshape(-1), **kw)
    keep = [0, 1, 3]
    ref = ctx.run_host([sid] * 3, [s.N] * 3, a0=a0[keep].reshape(-1),
                       **{k: (v[keep] if isinstance(v, np.ndarray) else v) for k, v in kw.items()})
    ctx.free_system(sid)
    nonfinite = gpu_status_bit("NONFINITE")
    assert g["status"][2] & nonfinite and g["steps"][2] == 1
    for i in keep:
        assert not g["status"][i] & nonfinite and g["steps"][i] == b.n_steps[i]
    P = g["P"].reshape(b.B, s.N)[keep]
    tol = 1e-13 if schedule == "queue" else 0.0
    assert np.max(np.abs(P - ref["P"].reshape(3, s.N))) <= tol


def gpu_status_bit(name):
    import paper_2312_02322_amd as mq
    return mq.STATUS[name]
