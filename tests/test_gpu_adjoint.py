"""GPU checks of the adjoint (backward-in-time) gradient of final probabilities.

L = sum_b sum_n w_bn P_b(n) for random weights w; the gradient with respect to
the 96 potential coefficients theta (two-rotor system, 12 angular terms x 8
radial functions) is checked against
  * central finite differences of GPU forward runs (h = 1e-6, relative 1e-5),
  * the FP64 oracle's forward-mode (dual-number) derivative of the same discrete
    RK4 map along random directions,
and is independent of the checkpoint interval.
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
def setup(gpu_lib):
    ctx = gpu_lib.Context()
    (s,), b = S.config4(n_traj=4, n_steps=300, jmax=2)
    sid = ctx.load_system(s)
    ctx.set_params(sid, s.param_radial, s.param_G_index, s.G)
    rng = np.random.default_rng(11)
    w = rng.standard_normal((b.B, s.N))
    yield ctx, sid, s, b, w
    ctx.synchronize()
    ctx.close()


def forward_L(ctx, sid, s, b, w, theta):
    ctx.set_theta(sid, theta)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                     b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps)
    return float(np.sum(w * g["P"].reshape(b.B, s.N))), g["P"].reshape(b.B, s.N)


def adjoint(ctx, sid, s, b, w, S_=64):
    ctx.set_theta(sid, s.theta)
    return ctx.adjoint(sid, s.N, w, init_channel=b.init_channel, E_coll=b.E_coll, b=b.b,
                       dt=b.dt, n_steps=b.n_steps, R0=b.R0, checkpoint_every=S_)


def test_set_theta_rebuilds_the_loaded_tables(setup, gpu_lib):
    ctx, sid, s, b, w = setup
    say("set_theta vs host-built tables N=%d" % s.N)
    L1, P1 = forward_L(ctx, sid, s, b, w, s.theta)
    sid2 = ctx.load_system(s)           # tables built on the host at the same theta
    g = ctx.run_host([sid2] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                     b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps)
    assert np.max(np.abs(g["P"].reshape(b.B, s.N) - P1)) < 1e-12
    ctx.free_system(sid2)


def test_adjoint_matches_central_differences(setup):
    ctx, sid, s, b, w = setup
    say("adjoint vs central differences N=%d B=%d steps=%d" % (s.N, b.B, b.n_steps[0]))
    grad, P = adjoint(ctx, sid, s, b, w)
    _, Pf = forward_L(ctx, sid, s, b, w, s.theta)
    assert np.max(np.abs(P - Pf)) < 1e-12
    h = 1e-6
    scale = np.max(np.abs(grad))
    for p in [0, 6, 7, 13, 30, 47, 55, 71, 88, 95]:
        e = np.zeros_like(s.theta); e[p] = h
        Lp, _ = forward_L(ctx, sid, s, b, w, s.theta + e)
        Lm, _ = forward_L(ctx, sid, s, b, w, s.theta - e)
        fd = (Lp - Lm) / (2 * h)
        say("  theta[%d]: adjoint %.10e  fd %.10e" % (p, grad[p], fd))
        assert abs(grad[p] - fd) <= 1e-5 * max(abs(fd), 1e-3 * scale)


def test_adjoint_matches_oracle_forward_mode(setup):
    ctx, sid, s, b, w = setup
    say("adjoint vs oracle forward mode")
    grad, _ = adjoint(ctx, sid, s, b, w)
    rng = np.random.default_rng(5)
    for _ in range(2):
        v = rng.standard_normal(s.theta.shape[0])
        o = oracle.OracleSystem(s, tangent_tables=S.parametric_tables(s, v))
        _, dP = o.tangent_rk4(b)
        dL = float(np.sum(w * dP))
        say("  direction: adjoint %.12e  oracle %.12e" % (grad @ v, dL))
        assert abs(grad @ v - dL) <= 1e-9 * max(abs(dL), 1e-12) + 1e-13


def test_checkpoint_interval_does_not_change_the_gradient(setup):
    ctx, sid, s, b, w = setup
    say("checkpoint intervals 1, 7, 300, 2^31-1")
    g1, _ = adjoint(ctx, sid, s, b, w, S_=1)
    g7, _ = adjoint(ctx, sid, s, b, w, S_=7)
    g300, _ = adjoint(ctx, sid, s, b, w, S_=300)
    # one segment: every stage state stored by the forward pass, nothing recomputed
    gall, _ = adjoint(ctx, sid, s, b, w, S_=2 ** 31 - 1)
    assert np.array_equal(g1, g7) and np.array_equal(g1, g300) and np.array_equal(g1, gall)


def test_ragged_step_counts_one_segment_and_checkpoints(setup):
    """Trajectories of 300, 150, 0 and 299 steps in one gradient: the one-segment form
    (a forward and a backward launch, every stage state stored) and the fused form with
    checkpoints every 7 steps give the same gradient and probabilities bit for bit, and
    the probabilities are those of the forward propagation."""
    ctx, sid, s, b, w = setup
    ctx.set_theta(sid, s.theta)
    ns = np.array([300, 150, 0, 299], np.int64)
    kw = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, dt=b.dt, n_steps=ns, R0=b.R0)
    say("ragged adjoint: steps %s" % ns.tolist())
    g1, P1 = ctx.adjoint(sid, s.N, w, checkpoint_every=2 ** 31 - 1, **kw)
    g7, P7 = ctx.adjoint(sid, s.N, w, checkpoint_every=7, **kw)
    assert np.array_equal(g1, g7) and np.array_equal(P1, P7)
    f = ctx.run_host([sid] * b.B, [s.N] * b.B, **kw)
    assert np.max(np.abs(P1.reshape(b.B, s.N) - f["P"].reshape(b.B, s.N))) < 1e-12
    assert np.all(P1.reshape(b.B, s.N)[2] == (np.arange(s.N) == b.init_channel[2]))


def test_autograd_function(setup):
    import torch
    import paper_2312_02322_amd as mq
    ctx, sid, s, b, w = setup
    say("torch.autograd through the adjoint")
    theta = torch.tensor(s.theta, dtype=torch.float64, requires_grad=True)
    batch = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                 n_steps=b.n_steps)
    P = mq.propagate(theta, ctx, sid, s.N, batch, checkpoint_every=64)
    L = (torch.as_tensor(w) * P).sum()
    L.backward()
    grad, _ = adjoint(ctx, sid, s, b, w)
    assert np.allclose(theta.grad.numpy(), grad, rtol=0, atol=1e-14 * np.max(np.abs(grad)))
