"""Device allocation failures, injected from the host (MQCT_FAULT=alloc fails
every allocation of the library, MQCT_FAULT=alloc@n only the n-th): each call
reports MQCT_ERR_OOM, frees what it had taken, and leaves the context usable.
No kernel is made to fail; only the allocation calls are refused."""
import os
import sys

import numpy as np
import pytest

from synth import systems as S

pytestmark = pytest.mark.gpu


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


class fault:
    def __init__(self, value):
        self.value = value

    def __enter__(self):
        os.environ["MQCT_FAULT"] = self.value

    def __exit__(self, *exc):
        os.environ.pop("MQCT_FAULT", None)


def test_allocation_failures_report_oom_and_free_what_they_took(gpu_lib):
    import torch
    ctx = gpu_lib.Context()
    (s,), b = S.config1(n_traj=8, n_steps=20, jmax=3)
    kw = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
              n_steps=b.n_steps)
    sid = ctx.load_system(s)
    ref = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="binned", **kw)
    ctx.free_system(sid)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(ctx.device)[0]

    with fault("alloc"):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.load_system(s)
    assert e.value.code == gpu_lib.ERR_OOM
    # every allocation of a dense and of a sparse load in turn
    for layout in ("dense", "sparse"):
        failed = 0
        for n in range(1, 64):
            with fault("alloc@%d" % n):
                try:
                    sid = ctx.load_system(s, layout=layout)
                except gpu_lib.MQCTError as err:
                    assert err.code == gpu_lib.ERR_OOM, err
                    failed += 1
                    continue
            ctx.free_system(sid)
            break
        say("  %s load: allocations 1..%d refused in turn, each reported as out of memory" % (
            layout, failed))
        assert failed >= 4
    # a run whose workspace must grow
    sid = ctx.load_system(s)
    big = 64
    bb = b.subset(np.arange(big) % b.B)
    kwb = dict(init_channel=bb.init_channel, E_coll=bb.E_coll, b=bb.b, R0=bb.R0, dt=bb.dt,
               n_steps=bb.n_steps)
    with fault("alloc"):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.run_host([sid] * big, [s.N] * big, schedule="binned", **kwb)
    assert e.value.code == gpu_lib.ERR_OOM
    g = ctx.run_host([sid] * b.B, [s.N] * b.B, schedule="binned", **kw)
    for k in ("P", "classical", "t_final", "steps", "status"):
        assert np.array_equal(g[k], ref[k]), k
    gb = ctx.run_host([sid] * big, [s.N] * big, schedule="binned", **kwb)
    assert np.array_equal(gb["P"].reshape(big, s.N)[:b.B], ref["P"].reshape(b.B, s.N))
    ctx.free_system(sid)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info(ctx.device)[0]
    say("  device memory free before %.1f MB, after %.1f MB (the run's workspace grew)" % (
        free0 / 1e6, free1 / 1e6))
    # what remains is the grown run workspace of the context, well under 256 MB
    assert free0 - free1 < 256e6
    ctx.close()
