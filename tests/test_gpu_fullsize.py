"""Full-size parity subsets of the workloads, against the FP64 oracle.

* N = 969 (asymmetric top + atom, 200 knots, RK4 steps of 12 a.u.): the four
  shortest of the 4096 full collisions of the workload, from the grid end until
  they leave it, on the binned and per-trajectory schedules; FP64 tables within
  1e-9 per channel, FP32 tables within 1e-4.
* N = 256 (two rotors, 96 potential coefficients, 1024 trajectories x 4096 RK4
  steps, the tables stored sparse as in the timed workload): the adjoint
  gradient of a b-weighted inelastic sum against central differences of GPU
  forward runs on every coefficient, and on 16 of the trajectories against the
  oracle's forward-mode (dual-number) derivative along random directions.
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


def start(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                n_steps=b.n_steps)


@pytest.fixture(scope="module")
def collisions969(gpu_lib):
    (s,), b = S.config2(n_traj=4096)
    pick = np.argsort(b.n_steps, kind="stable")[:4]
    sub = b.subset(pick)
    say("N=%d: trajectories %s, %s RK4 steps of %.0f a.u." % (s.N, pick.tolist(),
                                                              sub.n_steps.tolist(), sub.dt[0]))
    ref = oracle.OracleSystem(s).propagate(sub)
    say("  oracle done, status %s" % ref["status"].tolist())
    ctx = gpu_lib.Context()
    yield ctx, s, sub, ref
    ctx.close()


@pytest.mark.parametrize("storage,schedule", [("C128", "binned"), ("C128", "gemv"),
                                              ("C64", "binned"), ("C64", "gemv")])
def test_config2_full_collisions(collisions969, storage, schedule):
    ctx, s, b, ref = collisions969
    sid = ctx.load_system(s, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule=schedule, **start(b))
    ctx.free_system(sid)
    P = g["P"].reshape(b.B, s.N)
    d = np.max(np.abs(P - ref["P"]))
    dc = np.max(np.abs(g["classical"].reshape(b.B, 6) - ref["classical"]) /
                (1 + np.abs(ref["classical"])))
    say("  %s %s: max|dP| %.3e, classical %.3e, status %s" % (storage, schedule, d, dc,
                                                             g["status"].tolist()))
    assert np.array_equal(g["status"], ref["status"])
    assert np.array_equal(g["steps"], ref["steps"])
    assert d < (1e-9 if storage == "C128" else 1e-4)
    assert dc < (1e-9 if storage == "C128" else 1e-5)


@pytest.fixture(scope="module")
def gradient256(gpu_lib):
    (s,), b = S.config4()
    ctx = gpu_lib.Context()
    sid = ctx.load_system(s, layout="sparse")
    ctx.set_params(sid, s.param_radial, s.param_G_index, s.G)
    ctx.set_theta(sid, s.theta)
    lev = s.level_of_channel
    w = np.array([(2 * np.pi * b.b_max / b.B) * b.b[i] * (lev != b.init_level[i])
                  for i in range(b.B)])
    yield ctx, sid, s, b, w
    ctx.close()


def test_config4_gradient_against_central_differences(gradient256):
    ctx, sid, s, b, w = gradient256
    say("N=%d adjoint, %d trajectories x %d steps, %d coefficients" % (
        s.N, b.B, b.n_steps[0], s.theta.shape[0]))
    ctx.set_theta(sid, s.theta)
    grad, P = ctx.adjoint(sid, s.N, w, checkpoint_every=256, **start(b))

    def L_at(theta):
        ctx.set_theta(sid, theta)
        g = ctx.run_host([sid] * b.B, [s.N] * b.B, **start(b))
        return float(np.sum(w * g["P"].reshape(b.B, s.N)))

    h = 1e-6
    scale = np.max(np.abs(grad))
    worst = 0.0
    for p in range(s.theta.shape[0]):
        e = np.zeros_like(s.theta)
        e[p] = h
        fd = (L_at(s.theta + e) - L_at(s.theta - e)) / (2 * h)
        err = abs(grad[p] - fd) / max(abs(fd), 1e-3 * scale)
        worst = max(worst, err)
        if p % 8 == 0:
            say("  theta[%d]: adjoint %.10e fd %.10e" % (p, grad[p], fd))
        assert err <= 1e-5, (p, grad[p], fd)
    ctx.set_theta(sid, s.theta)
    say("  all %d coefficients within %.2e (relative)" % (s.theta.shape[0], worst))


def test_config4_gradient_against_oracle_forward_mode(gradient256):
    ctx, sid, s, b, w = gradient256
    sub = b.subset(np.arange(16))
    ws = w[:16]
    ctx.set_theta(sid, s.theta)
    grad, _ = ctx.adjoint(sid, s.N, ws, checkpoint_every=256, **start(sub))
    rng = np.random.default_rng(17)
    for _ in range(2):
        v = rng.standard_normal(s.theta.shape[0])
        o = oracle.OracleSystem(s, tangent_tables=S.parametric_tables(s, v))
        _, dP = o.tangent_rk4(sub)
        dL = float(np.sum(ws * dP))
        say("  16 trajectories x %d steps, direction: adjoint %.12e oracle %.12e" % (
            sub.n_steps[0], grad @ v, dL))
        assert abs(grad @ v - dL) <= 1e-9 * max(abs(dL), 1e-12) + 1e-13
