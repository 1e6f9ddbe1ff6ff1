"""GPU parity of the sparse (ELL) layout of the coupling tables.

The matrices of Eq. 5 follow angular-momentum selection rules: most of their
elements vanish at every R (92 % for the two-rotor system at j <= 3).  The
sparse layout stores, per column n, only the rows m whose element exceeds
drop_below somewhere on the grid; drop_below = 0 keeps every structural
nonzero, so the result is that of the dense tables.

* drop_below = 0 against the dense layout: bitwise on the per-trajectory
  schedule with FP64 tables (the same products in the same order, the zeros
  left out), 1e-12 on the work list (its split forms cut the rows elsewhere),
  1e-6 with FP32 tables (their partial sums are cut into other chunks);
* drop_below > 0 against the oracle run on tables truncated on the host with
  the same rule (kept if |M(m,n)| or |M(n,m)| exceeds it at some knot);
* complex Hermitian tables, DP5 on the work list, a batch mixing sparse and
  dense systems;
* the adjoint: sparse and dense gradients agree, and with truncation the
  gradient is that of the truncated model (central differences);
* the stored bytes shrink to the kept slots; the binned schedule and bad
  thresholds are refused.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S
from synth.systems import System

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


def kept_pattern(M, thr):
    A = np.abs(M).max(axis=0)
    return (A > thr) | (A.T > thr)


def with_tables(s, M, name):
    return System(name, s.R_grid, s.E, M, s.jx_row, s.jx_col, s.jx_val, s.mu,
                  s.level_of_channel, s.n_levels)


def truncated(s, thr):
    keep = kept_pattern(s.M, thr)
    return with_tables(s, np.where(keep[None], s.M, 0.0), "truncated"), keep


def gauge_complex(s, seed=3):
    """D M D^H with D = diag(exp(i phi_n)): Hermitian, complex, same pattern."""
    ph = np.exp(1j * np.random.default_rng(seed).uniform(0, 2 * np.pi, s.N))
    return with_tables(s, ph[None, :, None] * s.M * np.conj(ph)[None, None, :], "complex")


def run(ctx, sid, s, b, **kw):
    return ctx.run_host([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                        b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps, **kw)


def pair(ctx, s, storage=None, thr=0.0):
    return (ctx.load_system(s, storage=storage),
            ctx.load_system(s, storage=storage, layout="sparse", drop_below=thr))


def free(ctx, *ids):
    for i in ids:
        ctx.free_system(i)


@pytest.mark.parametrize("which", ["config1", "config4", "complex"])
def test_exact_pattern_equals_dense_fp64(ctx, which):
    if which == "config4":
        (s,), b = S.config4(n_traj=8, n_steps=200, jmax=3)
    else:
        (s,), b = S.config1(n_traj=8, n_steps=400, jmax=3)
        if which == "complex":
            s = gauge_complex(s)
    say("sparse(0) vs dense %s N=%d B=%d" % (which, s.N, b.B))
    d, sp = pair(ctx, s)
    for sched in ("gemv", "queue"):
        gd = run(ctx, d, s, b, schedule=sched)
        gs = run(ctx, sp, s, b, schedule=sched)
        err = np.max(np.abs(gd["P"] - gs["P"]))
        say("  %s max|dP| %.3e" % (sched, err))
        if sched == "gemv":
            assert np.array_equal(gd["P"], gs["P"])
            assert np.array_equal(gd["classical"], gs["classical"])
        else:
            assert err < 1e-12
            assert np.max(np.abs(gd["classical"] - gs["classical"]) /
                          (1 + np.abs(gd["classical"]))) < 1e-12
    free(ctx, d, sp)


@pytest.mark.parametrize("storage", ["R32", "C64"])
def test_exact_pattern_equals_dense_fp32(ctx, storage):
    (s,), b = S.config1(n_traj=8, n_steps=400, jmax=3)
    if storage == "C64":
        s = gauge_complex(s)
    say("sparse(0) vs dense, %s tables N=%d" % (storage, s.N))
    d, sp = pair(ctx, s, storage=storage)
    for sched in ("gemv", "queue"):
        gd = run(ctx, d, s, b, schedule=sched)
        gs = run(ctx, sp, s, b, schedule=sched)
        err = np.max(np.abs(gd["P"] - gs["P"]))
        say("  %s max|dP| %.3e" % (sched, err))
        assert err < 1e-6
    free(ctx, d, sp)


@pytest.mark.parametrize("which", ["config4", "complex"])
def test_truncated_tables_match_the_oracle(ctx, which):
    if which == "config4":
        (s,), b = S.config4(n_traj=4, n_steps=200, jmax=3)
        thr = 1e-3
    else:
        (s,), b = S.config1(n_traj=6, n_steps=400, jmax=3)
        s = gauge_complex(s)
        thr = 2e-3
    t, keep = truncated(s, thr)
    full = kept_pattern(s.M, 0.0)
    assert keep.sum() < full.sum()          # the threshold removes elements
    say("truncated %s N=%d: %d of %d elements kept" % (which, s.N, keep.sum(), full.sum()))
    sp = ctx.load_system(s, layout="sparse", drop_below=thr)
    o = oracle.OracleSystem(t).propagate(b)
    o_full = oracle.OracleSystem(s).propagate(b)
    for sched in ("gemv", "queue"):
        g = run(ctx, sp, s, b, schedule=sched)
        err = np.max(np.abs(g["P"].reshape(b.B, s.N) - o["P"]))
        say("  %s max|dP| vs truncated oracle %.3e, truncation effect %.3e" %
            (sched, err, np.max(np.abs(o["P"] - o_full["P"]))))
        assert err < 1e-9
        assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < 1e-10
    assert np.max(np.abs(o["P"] - o_full["P"])) > 1e-6   # the truncation is visible
    free(ctx, sp)


def test_dp5_sparse_equals_dense(ctx):
    (s,), b = S.config1(n_traj=6, n_steps=1, jmax=3)
    say("DP5 sparse vs dense N=%d" % s.N)
    d, sp = pair(ctx, s)
    kw = dict(integrator="dp5", rtol=1e-8, atol=1e-8, max_steps=50000, h_min=1e-6)
    gd = run(ctx, d, s, b, **kw)
    gs = run(ctx, sp, s, b, **kw)
    assert np.all(gd["status"] & 1) and np.all(gs["status"] & 1)
    assert np.max(np.abs(gd["steps"] - gs["steps"])) <= 2
    assert np.max(np.abs(gd["P"] - gs["P"])) < 1e-7
    free(ctx, d, sp)


def test_mixed_sparse_and_dense_systems_in_one_batch(ctx):
    (s1,), b1 = S.config1(n_traj=5, n_steps=300, jmax=3)
    (s4,), b4 = S.config4(n_traj=3, n_steps=300, jmax=3)
    say("mixed batch: N=%d dense + sparse, N=%d sparse" % (s1.N, s4.N))
    d1 = ctx.load_system(s1)
    p1 = ctx.load_system(s1, layout="sparse")
    p4 = ctx.load_system(s4, layout="sparse")
    sids = [d1] * b1.B + [p1] * b1.B + [p4] * b4.B
    Ns = [s1.N] * (2 * b1.B) + [s4.N] * b4.B
    cat = lambda f: np.concatenate([getattr(b1, f), getattr(b1, f), getattr(b4, f)])
    g = ctx.run_host(sids, Ns, schedule="queue", init_channel=cat("init_channel"),
                     E_coll=cat("E_coll"), b=cat("b"), R0=cat("R0"), dt=cat("dt"),
                     n_steps=cat("n_steps"))
    P = g["P"]
    n1 = b1.B * s1.N
    ref1 = run(ctx, d1, s1, b1, schedule="gemv")["P"]
    ref4 = run(ctx, p4, s4, b4, schedule="gemv")["P"]
    assert np.max(np.abs(P[:n1] - ref1)) < 1e-12
    assert np.max(np.abs(P[n1:2 * n1] - ref1)) < 1e-12
    assert np.max(np.abs(P[2 * n1:] - ref4)) < 1e-12
    free(ctx, d1, p1, p4)


def test_adjoint_sparse_equals_dense(ctx):
    (s,), b = S.config4(n_traj=4, n_steps=200, jmax=2)
    rng = np.random.default_rng(5)
    w = rng.standard_normal((b.B, s.N))
    say("adjoint sparse vs dense N=%d" % s.N)
    grads = []
    for layout in ("dense", "sparse"):
        sid = ctx.load_system(s, layout=layout)
        ctx.set_params(sid, s.param_radial, s.param_G_index, s.G)
        ctx.set_theta(sid, s.theta)
        grads.append(ctx.adjoint(sid, s.N, w, init_channel=b.init_channel, E_coll=b.E_coll,
                                 b=b.b, dt=b.dt, n_steps=b.n_steps, R0=b.R0,
                                 checkpoint_every=50))
        ctx.free_system(sid)
    (gd, Pd), (gs, Ps) = grads
    assert np.max(np.abs(Pd - Ps)) < 1e-12
    assert np.max(np.abs(gd - gs)) < 1e-10 * np.max(np.abs(gd))


def test_adjoint_of_truncated_tables_matches_central_differences(ctx):
    (s,), b = S.config4(n_traj=4, n_steps=200, jmax=2)
    A = np.sort(np.abs(s.M).max(axis=0)[kept_pattern(s.M, 0.0)])
    thr = float(A[len(A) // 4])             # drops about a quarter of the nonzeros
    rng = np.random.default_rng(6)
    w = rng.standard_normal((b.B, s.N))
    say("adjoint of truncated tables N=%d, drop_below %.3e" % (s.N, thr))
    sid = ctx.load_system(s, layout="sparse", drop_below=thr)
    ctx.set_params(sid, s.param_radial, s.param_G_index, s.G)
    ctx.set_theta(sid, s.theta)
    grad, P = ctx.adjoint(sid, s.N, w, init_channel=b.init_channel, E_coll=b.E_coll, b=b.b,
                          dt=b.dt, n_steps=b.n_steps, R0=b.R0, checkpoint_every=50)

    def L(theta):
        ctx.set_theta(sid, theta)
        return float(np.sum(w * run(ctx, sid, s, b)["P"].reshape(b.B, s.N)))

    h = 1e-6
    scale = np.max(np.abs(grad))
    for p in [0, 7, 13, 30, 55, 88]:
        e = np.zeros_like(s.theta)
        e[p] = h
        fd = (L(s.theta + e) - L(s.theta - e)) / (2 * h)
        say("  theta[%d]: adjoint %.10e  fd %.10e" % (p, grad[p], fd))
        assert abs(grad[p] - fd) <= 1e-5 * max(abs(fd), 1e-3 * scale)
    ctx.free_system(sid)


def test_stored_bytes_and_refusals(ctx, gpu_lib):
    (s,), b = S.config4(n_traj=4, n_steps=20, jmax=3)
    d, sp = pair(ctx, s)
    keep = kept_pattern(s.M, 0.0)
    W = int(keep.sum(axis=0).max())
    Npad = (s.N + 15) // 16 * 16
    say("stored bytes N=%d W=%d" % (s.N, W))
    assert ctx.system_bytes(sp) == 2 * s.K * W * Npad * 8
    assert ctx.system_bytes(sp) < ctx.system_bytes(d) * W / s.N * 1.01
    with pytest.raises(gpu_lib.MQCTError) as e:
        run(ctx, sp, s, b, schedule="binned")
    assert e.value.code == gpu_lib.ERR_UNSUPPORTED
    for bad in (-1.0, float("nan"), float("inf")):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.load_system(s, layout="sparse", drop_below=bad)
        assert e.value.code == gpu_lib.ERR_ARG
    free(ctx, d, sp)
