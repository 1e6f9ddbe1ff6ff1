"""Writes n4096_rk4_1000_steps.npz: the FP64 oracle's state after the first 1000
RK4 steps of two trajectories of the N = 4096 random-table workload (512
trajectories from 20 A, 10,000 steps of T/10,000 over the collision), for the
GPU parity test of that workload.  The oracle holds the tables only at the run
of knots the two trajectories cross (R >= 29.5 bohr), with the second
derivatives of the whole grid's natural spline taken through the generator's
rank-Q factors (oracle.rank_q_knot_tables); building them takes about 40 GB of
host memory, the propagation a few minutes on two cores.

    python tests/golden/make_n4096_reference.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle                       # noqa: E402
from synth import systems as S      # noqa: E402

STEPS = 1000
TRAJ = [0, 1]
R_MIN_BOHR = 29.5
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "n4096_rk4_1000_steps.npz")


def main():
    t0 = time.time()
    (s,), b = S.config5(n_traj=512, n_steps=10000, build_tables=False)
    phi, v, H, scale = S.gp_rank_factors(s)
    ks = np.where(s.R_grid >= R_MIN_BOHR)[0]
    print("N=%d, knots %d..%d (R %.2f..%.2f bohr), factors in %.0fs" % (
        s.N, ks[0], ks[-1], s.R_grid[ks[0]], s.R_grid[ks[-1]], time.time() - t0), flush=True)
    knots = oracle.rank_q_knot_tables(s.R_grid, phi, v, H, ks, scale)
    del H
    print("knot tables in %.0fs" % (time.time() - t0), flush=True)
    sub = b.subset(TRAJ)
    sub.n_steps[:] = STEPS
    o = oracle.OracleSystem(s, knots=knots)
    ref = o.propagate(sub)
    R_min = float(np.min(ref["classical"][:, 0]))
    print("propagated in %.0fs, R down to %.3f bohr" % (time.time() - t0, R_min), flush=True)
    # the interval lookup of the last step stays inside the run of knots
    assert R_min > s.R_grid[ks[0]] and np.all(ref["status"] == 0)
    np.savez(OUT, traj=np.array(TRAJ), steps=STEPS, knots=ks, P=ref["P"],
             classical=ref["classical"], t_final=ref["t_final"], a_final=ref["a_final"])
    print("wrote", OUT)


if __name__ == "__main__":
    main()
