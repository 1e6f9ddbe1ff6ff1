"""The large workload at full size against the oracle: N = 4096 random Hermitian
tables on the 200-knot grid (53.7 GB as complex FP32 values and curvatures, 107 GB
in FP64), all 512 trajectories of the workload on the binned schedule for the
first 1000 RK4 steps of their collision (R from 37.8 to about 30 bohr), two of
them against the FP64 oracle's state at that point (tests/golden/
n4096_rk4_1000_steps.npz, written by make_n4096_reference.py beside it: the
oracle on the run of knots they cross, its second derivatives those of the whole
grid's spline).  FP64 tables within 1e-9 per channel, FP32 tables within 1e-4.
"""
import os
import sys

import numpy as np
import pytest

from synth import systems as S

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "n4096_rk4_1000_steps.npz")


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def large(gpu_lib):
    ref = np.load(GOLDEN)
    (s,), b = S.config5(n_traj=512, n_steps=10000, build_tables=False)
    b.n_steps[:] = int(ref["steps"])
    ctx = gpu_lib.Context()
    Md = S.gp_tables_device(s, ctx.device)
    say("N=%d tables built on the device; reference: trajectories %s x %d steps" % (
        s.N, ref["traj"].tolist(), int(ref["steps"])))
    yield ctx, s, b, Md, ref
    del Md
    ctx.close()


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_large_binned_first_steps_against_oracle(large, storage):
    ctx, s, b, Md, ref = large
    steps = int(ref["steps"])
    say("N=4096 %s binned: 512 trajectories x %d steps" % (storage, steps))
    sid = ctx.load_system(R_grid=s.R_grid, E=s.E, M=Md, jx=None, mu=s.mu, storage=storage)
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll,
                     b=b.b, R0=b.R0, dt=b.dt, n_steps=b.n_steps, schedule="binned")
    ctx.free_system(sid)
    tr = ref["traj"]
    P = g["P"].reshape(b.B, s.N)[tr]
    d = np.max(np.abs(P - ref["P"]))
    dc = np.max(np.abs(g["classical"].reshape(b.B, 6)[tr] - ref["classical"]) /
                (1 + np.abs(ref["classical"])))
    say("  max|dP| = %.3e, classical %.3e, max|norm-1| over the batch %.2e" % (
        d, dc, np.max(np.abs(g["norm_err"]))))
    assert np.all(g["status"] == 0) and np.all(g["steps"] == steps)
    assert d < (1e-9 if storage == "C128" else 1e-4)
    assert dc < (1e-9 if storage == "C128" else 1e-6)
