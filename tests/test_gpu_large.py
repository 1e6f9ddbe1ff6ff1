"""The large workload at full size against the oracle: N = 4096 random Hermitian
tables on the 200-knot grid (53.7 GB as complex FP32 values and curvatures, 107 GB
in FP64), all 512 trajectories of the workload on the binned schedule for the
first 100 RK4 steps of their collision, two of them propagated by the FP64 oracle
on the knots they touch (its second derivatives are those of the whole grid's
spline, taken through the generator's rank-Q factors).  FP64 tables within 1e-9
per channel, FP32 tables within 1e-4.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S

pytestmark = pytest.mark.gpu

STEPS = 100


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def large(gpu_lib):
    (s,), b = S.config5(n_traj=512, n_steps=10000, build_tables=False)
    b.n_steps[:] = STEPS
    ctx = gpu_lib.Context()
    Md = S.gp_tables_device(s, ctx.device)
    say("N=%d tables built on the device" % s.N)
    # the oracle's two trajectories, on the knots of the first hundred steps
    phi, v, H, scale = S.gp_rank_factors(s)
    ks = np.arange(s.K - 10, s.K)
    sub = b.subset([0, 1])
    o = oracle.OracleSystem(s, knots=oracle.rank_q_knot_tables(s.R_grid, phi, v, H, ks, scale))
    ref = o.propagate(sub)
    assert np.all(ref["classical"][:, 0] > s.R_grid[ks[0]]) and np.all(ref["status"] == 0)
    say("oracle: 2 trajectories x %d steps, R down to %.2f bohr" % (STEPS, ref["classical"][:, 0].min()))
    yield ctx, s, b, Md, ref
    del Md
    ctx.close()


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_large_binned_first_steps_against_oracle(large, storage):
    ctx, s, b, Md, ref = large
    say("N=4096 %s binned: 512 trajectories x %d steps" % (storage, STEPS))
    sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                     b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps, schedule="binned")
    ctx.free_system(sid)
    P = g["P"].reshape(b.B, s.N)[:2]
    d = np.max(np.abs(P - ref["P"]))
    dc = np.max(np.abs(g["classical"].reshape(b.B, 6)[:2] - ref["classical"]) /
                (1 + np.abs(ref["classical"])))
    say("  max|dP| = %.3e, classical %.3e, max|norm-1| over the batch %.2e" % (
        d, dc, np.max(np.abs(g["norm_err"]))))
    assert np.all(g["status"] == 0) and np.all(g["steps"] == STEPS)
    assert d < (1e-9 if storage == "C128" else 1e-4)
    assert dc < (1e-9 if storage == "C128" else 1e-6)
