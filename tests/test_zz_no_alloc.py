"""mqct_run_noalloc: the per-trajectory RK4 entry point that allocates no device
memory (its records and start amplitudes go to the library's static scratch
array).  Through the C ABI, two calls in a row -- the second with a smaller
batch, so the scratch holds the first call's contents when the second starts --
against mqct_run on the same schedule: the same kernels, so every result agrees
bit for bit."""
import sys

import numpy as np
import pytest

from synth import systems as S

pytestmark = pytest.mark.gpu

KEYS = ("P", "a_final", "classical", "t_final", "steps", "rejects", "status", "norm_err",
        "energy_err", "angmom_err")


def say(msg):
    print("[gpu] " + msg, flush=True)
    sys.stdout.flush()


def device_out(torch, dev, B, total):
    return {"P": torch.full((total,), -1.0, dtype=torch.float64, device=dev),
            "a_final": torch.zeros(total, dtype=torch.complex128, device=dev),
            "classical": torch.zeros((B, 6), dtype=torch.float64, device=dev),
            "t_final": torch.zeros(B, dtype=torch.float64, device=dev),
            "steps": torch.zeros(B, dtype=torch.int64, device=dev),
            "rejects": torch.zeros(B, dtype=torch.int64, device=dev),
            "status": torch.zeros(B, dtype=torch.int32, device=dev),
            "norm_err": torch.zeros(B, dtype=torch.float64, device=dev),
            "energy_err": torch.zeros(B, dtype=torch.float64, device=dev),
            "angmom_err": torch.zeros(B, dtype=torch.float64, device=dev)}


def test_noalloc_equals_run_on_two_calls(gpu_lib):
    import torch
    ctx = gpu_lib.Context()
    dev = ctx.device
    # a real (R64) and a complex FP32 (C64) system in one batch, records of both kinds
    (s1,), b1 = S.config1(n_traj=40, n_steps=150, jmax=4)
    (s2,), b2 = S.config2(n_traj=24, jmax=2)
    b2.n_steps[:] = 120
    id1 = ctx.load_system(s1, storage="R64")
    id2 = ctx.load_system(s2, storage="C64")
    rng = np.random.default_rng(7)
    for call, (n1, n2, with_a0) in enumerate(((40, 24, False), (9, 5, True))):
        order = rng.permutation(n1 + n2)
        ids = np.concatenate([np.full(n1, id1), np.full(n2, id2)])[order]
        Ns = np.concatenate([np.full(n1, s1.N), np.full(n2, s2.N)])[order]
        cat = lambda x, y: np.concatenate([np.asarray(x)[:n1], np.asarray(y)[:n2]])[order]
        kw = dict(E_coll=cat(b1.E_coll, b2.E_coll), b=cat(b1.b, b2.b), R0=cat(b1.R0, b2.R0),
                  dt=cat(b1.dt, b2.dt), n_steps=cat(b1.n_steps, b2.n_steps))
        if with_a0:
            a0 = np.zeros(int(Ns.sum()), np.complex128)
            offs = np.concatenate([[0], np.cumsum(Ns)])
            for i in range(len(Ns)):
                v = rng.standard_normal(Ns[i]) + 1j * rng.standard_normal(Ns[i])
                a0[offs[i]:offs[i + 1]] = v / np.linalg.norm(v)
            kw["a0"] = a0
        else:
            kw["init_channel"] = cat(b1.init_channel, b2.init_channel)
        B, total = len(ids), int(Ns.sum())
        say("call %d: %d trajectories (N=%d and %d), a0 %s" % (call + 1, B, s1.N, s2.N, with_a0))
        ref = ctx.run(ids, Ns, schedule="gemv", **kw)
        torch.cuda.synchronize()
        out = device_out(torch, dev, B, total)
        free0 = torch.cuda.mem_get_info(dev)[0]
        ctx.run_noalloc(ids, out, **kw)
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info(dev)[0]
        assert free1 >= free0, "the no-allocation entry point took device memory"
        for k in KEYS:
            assert torch.equal(out[k], ref[k]), k
        assert np.all(out["steps"].cpu().numpy() == kw["n_steps"])
    # beyond the scratch: refused before any device work
    big = 90000
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.run_noalloc(np.full(big, id1, np.int32), device_out(torch, dev, 1, 1),
                        init_channel=np.zeros(big, np.int32), E_coll=np.full(big, 1e-3),
                        b=np.zeros(big), dt=np.full(big, 10.0), n_steps=np.zeros(big, np.int64))
    assert e.value.code == gpu_lib.ERR_ARG
    with pytest.raises(gpu_lib.MQCTError) as e:      # not the per-trajectory RK4 path
        lib = gpu_lib.lib()
        bd = gpu_lib.BatchDesc()
        bd.B = 1
        bd.integrator = 1
        res = gpu_lib.BatchResult()
        res.mem = gpu_lib.MEM_DEVICE
        res.P = 1
        ctx._check(lib.mqct_run_noalloc(ctx.h, gpu_lib.C.byref(bd), gpu_lib.C.byref(res)))
    assert e.value.code == gpu_lib.ERR_UNSUPPORTED
    ctx.free_system(id1)
    ctx.free_system(id2)
    ctx.close()
