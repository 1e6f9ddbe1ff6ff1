"""The trajectory state store (mqct_get_state / mqct_set_state, resume = 1).

A run split in two -- the first part's final states copied to the host with
get_state, written back with set_state, the second part continued with resume
-- must equal the uninterrupted run bit for bit (the state of Section II's
equations plus what the steppers carry: time, step size, rejection flag, counts,
status, the references of the diagnostics), for fixed-step RK4 and adaptive DP5
on every schedule that runs them.
"""
import sys

import numpy as np
import pytest

from synth import systems as S

pytestmark = pytest.mark.gpu

FIELDS = ("P", "a_final", "classical", "t_final", "steps", "rejects", "status", "norm_err",
          "energy_err", "angmom_err")


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def ctx(gpu_lib):
    c = gpu_lib.Context()
    c.set_option("tail", 0)        # one workgroup shape per class throughout
    yield c
    c.synchronize()
    c.close()


def start_args(b):
    return dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)


def assert_same(x, y):
    for f in FIELDS:
        if not np.array_equal(x[f], y[f]):
            say("  %s differs: %s vs %s" % (f, np.asarray(x[f]).ravel()[:8], np.asarray(y[f]).ravel()[:8]))
            say("  steps %s vs %s, status %s vs %s, t %s vs %s" % (
                x["steps"], y["steps"], x["status"], y["status"], x["t_final"], y["t_final"]))
        assert np.array_equal(x[f], y[f]), f


def round_trip(ctx):
    """The stored states through host memory and back."""
    rec, amps = ctx.get_state()
    ctx.set_state(rec.copy(), amps.copy())
    return rec, amps


@pytest.mark.parametrize("schedule", ["gemv", "queue", "binned"])
def test_rk4_split_run_equals_whole_run(ctx, schedule):
    (s,), b = S.config1(n_traj=6, n_steps=300, jmax=3)
    say("RK4 split 120 + 180 steps vs 300, N=%d, %s schedule" % (s.N, schedule))
    sid = ctx.load_system(s)
    ids, Ns = [sid] * b.B, [s.N] * b.B
    whole = ctx.run_host(ids, Ns, dt=b.dt, n_steps=b.n_steps, schedule=schedule, **start_args(b))
    ctx.run_host(ids, Ns, dt=b.dt, n_steps=np.full(b.B, 120), schedule=schedule, **start_args(b))
    rec, amps = round_trip(ctx)
    assert np.all(rec["steps"] == 120) and np.all(rec["n_origin"] == 120)
    assert np.array_equal(rec["h"], b.dt) and np.all(rec["t_origin"] == 0.0)
    rest = ctx.run_host(ids, Ns, n_steps=np.full(b.B, 180), schedule=schedule, resume=True)
    assert_same(rest, whole)
    # the store now holds the end of the whole run
    rec2, amps2 = ctx.get_state()
    assert np.array_equal(amps2, whole["a_final"])
    assert np.array_equal(rec2["t"], whole["t_final"]) and np.all(rec2["steps"] == 300)
    assert np.array_equal(rec2["classical"], whole["classical"].reshape(b.B, 6))
    ctx.free_system(sid)


@pytest.mark.parametrize("schedule", ["queue", "binned"])
def test_dp5_split_run_equals_whole_run(ctx, schedule):
    """Stopped by the accepted-step limit, continued with a larger one: the step
    size, the no-growth-after-rejection flag and the counts carry over, and the
    first stage is re-evaluated at the stored state (first same as last)."""
    (s,), b = S.config1(n_traj=6, n_steps=1, jmax=3)
    say("DP5 split at 25 accepted steps vs whole, N=%d, %s schedule" % (s.N, schedule))
    sid = ctx.load_system(s)
    ids, Ns = [sid] * b.B, [s.N] * b.B
    kw = dict(integrator="dp5", rtol=1e-8, atol=1e-8, schedule=schedule)
    whole = ctx.run_host(ids, Ns, max_steps=100000, **kw, **start_args(b))
    assert np.all(whole["status"] & 1) and np.all(whole["steps"] > 40)
    part = ctx.run_host(ids, Ns, max_steps=25, **kw, **start_args(b))
    assert np.all(part["status"] & 2) and np.all(part["steps"] == 25)
    rec, _ = round_trip(ctx)
    assert np.all(rec["t_origin"] == rec["t"]) and np.all(rec["h"] > 0)
    rest = ctx.run_host(ids, Ns, max_steps=100000, resume=True, **kw)
    assert_same(rest, whole)
    # exited trajectories are returned unchanged by a further resume
    again = ctx.run_host(ids, Ns, max_steps=100000, resume=True, **kw)
    assert_same(again, whole)
    ctx.free_system(sid)


def test_store_redefined_in_a_new_context(gpu_lib):
    """set_state with a new count defines the store, so a run can continue in
    another context (deterministic per-trajectory schedule: bit for bit)."""
    (s,), b = S.config1(n_traj=4, n_steps=200, jmax=2)
    c1 = gpu_lib.Context()
    sid = c1.load_system(s)
    ids, Ns = [sid] * b.B, [s.N] * b.B
    whole = c1.run_host(ids, Ns, dt=b.dt, n_steps=b.n_steps, schedule="gemv", **start_args(b))
    c1.run_host(ids, Ns, dt=b.dt, n_steps=np.full(b.B, 77), schedule="gemv", **start_args(b))
    rec, amps = c1.get_state()
    c1.close()
    c2 = gpu_lib.Context()
    sid2 = c2.load_system(s)
    assert c2.stored_count() == 0
    rec["system_id"] = sid2
    c2.set_state(rec, amps)
    assert c2.stored_count() == b.B
    rest = c2.run_host([sid2] * b.B, Ns, n_steps=np.full(b.B, 123), schedule="gemv", resume=True)
    assert_same(rest, whole)
    # a stored range can be overwritten in place (same systems)
    sub_rec, sub_amps = c2.get_state(1, 2)
    c2.set_state(sub_rec, sub_amps, first=1)
    c2.close()


def test_state_errors(ctx, gpu_lib):
    (s,), b = S.config1(n_traj=3, n_steps=5, jmax=1)
    sid = ctx.load_system(s)
    ids, Ns = [sid] * b.B, [s.N] * b.B
    ctx.run_host(ids, Ns, dt=b.dt, n_steps=b.n_steps, **start_args(b))
    assert ctx.stored_count() == 3
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.get_state(2, 5)
    assert e.value.code == gpu_lib.ERR_ARG
    with pytest.raises(gpu_lib.MQCTError) as e:      # B differs from the store
        ctx.run_host(ids[:2], Ns[:2], n_steps=[1, 1], resume=True)
    assert e.value.code == gpu_lib.ERR_STATE
    rec, amps = ctx.get_state()
    bad = rec.copy()
    bad["classical"][0, 0] = np.nan
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.set_state(bad, amps)
    assert e.value.code == gpu_lib.ERR_NONFINITE
    bad = rec.copy()
    bad["N"][1] += 1
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.set_state(bad, np.concatenate([amps, [0j]]))
    assert e.value.code == gpu_lib.ERR_ARG
    bad = rec.copy()
    bad["system_id"][0] = 999
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.set_state(bad, amps)
    assert e.value.code == gpu_lib.ERR_STATE
    ctx.free_system(sid)
