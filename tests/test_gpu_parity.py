"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars: FP64 tables, fixed-step RK4 -> final probabilities within 1e-9 of the
oracle (the two differ only in summation order, ~1e-13); FP32 tables -> within
1e-4.  Closed forms (Rabi, frozen-trajectory expm, free rotation) are checked
directly on the GPU as well.
"""
import math
import sys

import numpy as np
import pytest

import oracle
from synth import systems as S, units as U
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


def run_gpu(ctx, sid, system, batch, **kw):
    B = batch.B if batch is not None else len(kw["E_coll"])
    args = dict(init_channel=batch.init_channel, E_coll=batch.E_coll, b=batch.b, R0=batch.R0,
                dt=batch.dt, n_steps=batch.n_steps) if batch is not None else {}
    args.update(kw)
    out = ctx.run_host([sid] * B, [system.N] * B, **args)
    out["P"] = out["P"].reshape(B, system.N)
    out["a_final"] = out["a_final"].reshape(B, system.N)
    return out


def make_system(R, E, M, jx=None, mu=1000.0):
    N = len(E)
    if jx is None:
        jr = jc = np.zeros(0, np.int32); jv = np.zeros(0)
    else:
        jr, jc, jv = (np.asarray(jx[0], np.int32), np.asarray(jx[1], np.int32),
                      np.asarray(jx[2], np.float64))
    return System("test", np.asarray(R, float), np.asarray(E, float), M, jr, jc, jv, float(mu),
                  np.arange(N, dtype=np.int32), N)


# ------------------------------------------------------------------ stock configuration 1

def test_config1_full_batch_fp64(ctx):
    (s,), b = S.config1()
    say("config1 N=49 B=64 RK4 2000 steps R64")
    sid = ctx.load_system(s, storage="R64")
    g = run_gpu(ctx, sid, s, b)
    o = oracle.OracleSystem(s).propagate(b)
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    assert np.max(np.abs(g["a_final"] - o["a_final"])) < 1e-9
    assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < 1e-9
    assert np.array_equal(g["steps"], b.n_steps) and np.all(g["status"] == 0)
    assert np.max(np.abs(g["norm_err"] - o["norm_err"])) < 1e-9
    assert np.max(np.abs(g["energy_err"] - o["energy_err"])) < 1e-9
    assert np.max(np.abs(g["angmom_err"] - o["angmom_err"])) < 1e-9
    ctx.free_system(sid)


def test_config1_fp32_tables(ctx):
    (s,), b = S.config1()
    say("config1 N=49 B=64 R32 tables")
    sid = ctx.load_system(s, storage="R32")
    g = run_gpu(ctx, sid, s, b)
    o = oracle.OracleSystem(s).propagate(b)
    err = np.abs(g["P"] - o["P"])
    say("config1 fp32 max|dP| = %.3e" % err.max())
    assert err.max() < 1e-4
    ctx.free_system(sid)


# ------------------------------------------------------------------ closed forms on the GPU

def test_gpu_rabi_closed_form(ctx):
    Delta, V = 0.02, 0.015
    R = np.linspace(4.0, 40.0, 30)
    M = np.zeros((30, 2, 2)); M[:, 0, 1] = M[:, 1, 0] = V
    s = make_system(R, [0.0, Delta], M)
    say("rabi N=2")
    sid = ctx.load_system(s)
    Om = math.sqrt(Delta ** 2 + 4 * V ** 2)
    T, n = 700.0, 4000
    g = ctx.run_host([sid], [2], init_channel=[0], E_coll=[1e-3], b=[0.0], R0=[30.0],
                     dt=[T / n], n_steps=[n])
    assert abs(g["P"][1] - 4 * V ** 2 / Om ** 2 * math.sin(Om * T / 2) ** 2) < 1e-10
    ctx.free_system(sid)


def test_gpu_frozen_trajectory_expm(ctx):
    from scipy.linalg import expm
    rng = np.random.default_rng(7)
    N, K = 5, 20
    R = np.linspace(4.0, 24.0, K)
    E = np.sort(rng.uniform(0.0, 0.03, N))
    X = rng.standard_normal((K, N, N)) + 1j * rng.standard_normal((K, N, N))
    M = 0.01 * (X + np.conj(np.swapaxes(X, 1, 2))) / 2
    s = make_system(R, E, M, mu=1e30)
    say("frozen expm N=5 C128")
    sid = ctx.load_system(s)
    T, n = 300.0, 6000
    g = ctx.run_host([sid], [N], init_channel=[1], E_coll=[1e-3], b=[0.0], R0=[R[9]], dt=[T / n],
                     n_steps=[n])
    b0 = np.zeros(N, complex); b0[1] = 1
    aT = np.exp(1j * E * T) * (expm(-1j * (np.diag(E) + M[9]) * T) @ b0)
    assert np.max(np.abs(g["a_final"] - aT)) < 1e-10
    ctx.free_system(sid)


def test_gpu_free_rotation_wigner(ctx):
    from test_oracle_pins import wigner_small_d
    (s1,), _ = S.config1(n_traj=1, jmax=3)
    s = make_system(s1.R_grid, s1.E, np.zeros_like(s1.M), jx=(s1.jx_row, s1.jx_col, s1.jx_val),
                    mu=s1.mu)
    say("free rotation N=16 R64")
    sid = ctx.load_system(s)
    U_ = U.cm_to_hartree(500.0)
    bpar, R0 = 6.0, s.R_grid[-1]
    v = math.sqrt(2 * U_ / s.mu)
    s0 = math.sqrt(R0 ** 2 - bpar ** 2)
    T = 1.3 * s0 / v
    g = ctx.run_host([sid], [s.N], init_channel=[11], E_coll=[U_], b=[bpar], R0=[R0],
                     dt=[T / 4000], n_steps=[4000])
    Ph = math.atan2(bpar, s0 - v * T) - math.atan2(bpar, s0)
    assert abs(g["classical"][0, 2] - Ph) < 1e-10
    for idx in range(9, 16):
        assert abs(g["P"][idx] - wigner_small_d(3, s1.labels["m"][idx], -1, Ph) ** 2) < 1e-10
    ctx.free_system(sid)


# ------------------------------------------------------------------ complex tables, several tiles

def test_config2_reduced_fp64_and_fp32(ctx):
    """Asymmetric top j <= 3 (N = 84: several 16-column tiles and a ragged tail)."""
    (s,), b = S.config2(n_traj=6, jmax=3)
    b.n_steps[:] = np.minimum(b.n_steps, 3000)
    say("config2 reduced N=84 C128/C64, 6 trajectories")
    o = oracle.OracleSystem(s).propagate(b)
    sid = ctx.load_system(s, storage="C128")
    g = run_gpu(ctx, sid, s, b)
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    assert np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"]))) < 1e-9
    ctx.free_system(sid)
    sid = ctx.load_system(s, storage="C64")
    g = run_gpu(ctx, sid, s, b)
    err = np.abs(g["P"] - o["P"]).max()
    say("config2 reduced fp32 max|dP| = %.3e" % err)
    assert err < 1e-4
    ctx.free_system(sid)


def test_config4_rotor_rotor_fp64(ctx):
    (s,), b = S.config4(n_traj=4, n_steps=600)
    say("config4 N=256 R64 4 trajectories 600 steps")
    o = oracle.OracleSystem(s).propagate(b)
    sid = ctx.load_system(s)
    g = run_gpu(ctx, sid, s, b)
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    ctx.free_system(sid)


# ------------------------------------------------------------------ batching semantics

def test_mixed_systems_in_one_batch(ctx):
    """Ragged batch: two systems of different N (and dtype) interleaved."""
    (s1,), b1 = S.config1(n_traj=3, n_steps=300, jmax=4)
    (s2,), b2 = S.config2(n_traj=3, jmax=2)
    b2.n_steps[:] = 300
    say("mixed batch N=25 R64 + N=35 C128")
    id1 = ctx.load_system(s1)
    id2 = ctx.load_system(s2)
    order = [0, 3, 1, 4, 2, 5]
    sys_ids = np.array([id1] * 3 + [id2] * 3)[order]
    Ns = np.array([s1.N] * 3 + [s2.N] * 3)[order]
    cat = lambda a, c: np.concatenate([a, c])[order]
    g = ctx.run_host(sys_ids, Ns, init_channel=cat(b1.init_channel, b2.init_channel),
                     E_coll=cat(b1.E_coll, b2.E_coll), b=cat(b1.b, b2.b), R0=cat(b1.R0, b2.R0),
                     dt=cat(b1.dt, b2.dt), n_steps=cat(b1.n_steps, b2.n_steps))
    o1 = oracle.OracleSystem(s1).propagate(b1)["P"]
    o2 = oracle.OracleSystem(s2).propagate(b2)["P"]
    offs = np.concatenate([[0], np.cumsum(Ns)])
    for pos, src in enumerate(order):
        ref = o1[src] if src < 3 else o2[src - 3]
        assert np.max(np.abs(g["P"][offs[pos]:offs[pos + 1]] - ref)) < 1e-9
    ctx.free_system(id1)
    ctx.free_system(id2)


def test_resume_and_sharding_are_bitwise(ctx):
    (s,), b = S.config1(n_traj=8, n_steps=400)
    say("resume / shard N=49")
    sid = ctx.load_system(s)
    full = run_gpu(ctx, sid, s, b)
    again = run_gpu(ctx, sid, s, b)
    assert np.array_equal(full["a_final"], again["a_final"])          # deterministic
    half = b.subset(range(8)); half.n_steps[:] = 150
    first = run_gpu(ctx, sid, s, half)
    rest = run_gpu(ctx, sid, s, None, init_channel=None, a0=first["a_final"].reshape(-1),
                   classical0=first["classical"], t0=first["t_final"], dt=b.dt,
                   n_steps=np.full(8, 250), E_coll=b.E_coll)
    assert np.max(np.abs(rest["a_final"] - full["a_final"])) < 1e-12
    parts = [run_gpu(ctx, sid, s, b.subset(ix)) for ix in ([0, 1, 2], [3, 4, 5, 6, 7])]
    assert np.array_equal(np.concatenate([p["a_final"] for p in parts]), full["a_final"])
    ctx.free_system(sid)


def test_edge_cases(ctx, gpu_lib):
    (s,), b = S.config1(n_traj=2, n_steps=10, jmax=1)
    say("edge cases N=4")
    sid = ctx.load_system(s)
    z = run_gpu(ctx, sid, s, b, n_steps=[0, 0])
    assert np.array_equal(z["P"], np.eye(s.N)[b.init_channel])
    assert np.all(z["steps"] == 0) and np.allclose(z["classical"][:, 0], b.R0)
    # empty batch is a no-op
    ctx.run_host(np.zeros(0, np.int32), np.zeros(0, np.int64), init_channel=[], E_coll=[], b=[],
                 dt=[], n_steps=[])
    # invalid inputs are rejected before any device work
    with pytest.raises(gpu_lib.MQCTError) as e:
        run_gpu(ctx, sid, s, b, b=[100.0, 100.0])
    assert e.value.code == gpu_lib.ERR_ARG
    with pytest.raises(gpu_lib.MQCTError) as e:
        run_gpu(ctx, sid, s, b, init_channel=[0, 99])
    assert e.value.code == gpu_lib.ERR_ARG
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.run_host([sid + 7], [s.N], init_channel=[0], E_coll=[1e-3], b=[0.0], dt=[1.0],
                     n_steps=[1])
    assert e.value.code == gpu_lib.ERR_STATE
    bad = s.M.copy(); bad[3, 0, 1] = np.nan
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.load_system(make_system(s.R_grid, s.E, bad, mu=s.mu))
    assert e.value.code == gpu_lib.ERR_NONFINITE
    bad = s.M.copy(); bad[3, 0, 1] += 1e-3
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.load_system(make_system(s.R_grid, s.E, bad, mu=s.mu))
    assert e.value.code == gpu_lib.ERR_NOT_HERMITIAN
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.load_system(make_system(s.R_grid[::-1].copy(), s.E, s.M, mu=s.mu))
    assert e.value.code == gpu_lib.ERR_ARG
    ctx.free_system(sid)


def test_below_grid_flag(ctx):
    """A head-on trajectory on a grid that starts inside the wall is flagged."""
    (s,), b = S.config1(n_traj=1, n_steps=2000, jmax=2)
    k0 = np.searchsorted(s.labels["R_ang"], 3.6)
    cut = make_system(s.R_grid[k0:].copy(), s.E, s.M[k0:].copy(),
                      jx=(s.jx_row, s.jx_col, s.jx_val), mu=s.mu)
    say("below grid N=9")
    sid = ctx.load_system(cut)
    g = run_gpu(ctx, sid, cut, b, b=[0.0], E_coll=[U.cm_to_hartree(3000.0)])
    o = oracle.OracleSystem(cut).propagate(b, b=[0.0], E_coll=[U.cm_to_hartree(3000.0)])
    assert g["status"][0] & 8 and o["status"][0] & 8
    assert np.max(np.abs(g["P"] - o["P"])) < 1e-9
    ctx.free_system(sid)


def test_cross_sections_on_device(ctx):
    import torch
    (s,), b = S.config1(n_traj=64, n_steps=200)
    say("cross sections N=49 B=64")
    sid = ctx.load_system(s)
    out = ctx.run([sid] * b.B, [s.N] * b.B, init_channel=b.init_channel, E_coll=b.E_coll, b=b.b,
                  R0=b.R0, dt=b.dt, n_steps=b.n_steps)
    sig = ctx.cross_sections(out["P"].reshape(b.B, s.N), b.b, b.init_level,
                             s.level_of_channel, s.n_levels, b.b_max)
    torch.cuda.synchronize()
    P = out["P"].reshape(b.B, s.N).cpu().numpy()
    ref = oracle.cross_sections(b.init_level, b.b, P, s.level_of_channel, s.n_levels, b.b_max)
    assert np.max(np.abs(sig.cpu().numpy() - ref)) <= 1e-12 * np.max(np.abs(ref))
    ctx.free_system(sid)


def test_unsupported_combinations_report_cleanly(ctx, gpu_lib):
    """Two systems in one batch on the binned schedule (its products multiply one
    system's tables), sparse tables there, and an unknown schedule fail before any
    launch."""
    (s,), b = S.config1(n_traj=2, n_steps=10, jmax=1)
    sid = ctx.load_system(s)
    sid2 = ctx.load_system(s)
    sps = ctx.load_system(s, layout="sparse")
    common = dict(init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0)
    for ids, integ in (([sid, sid2], "dp5"), ([sid, sid2], "rk4"), ([sps, sps], "dp5")):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.run_host(ids, [s.N] * 2, integrator=integ, schedule="binned", dt=b.dt,
                         n_steps=b.n_steps, **common)
        assert e.value.code == gpu_lib.ERR_UNSUPPORTED
    ctx.free_system(sid2)
    ctx.free_system(sps)
    gpu_lib.SCHEDULES["bogus"] = 7
    try:
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.run_host([sid] * 2, [s.N] * 2, schedule="bogus", dt=b.dt, n_steps=b.n_steps,
                         **common)
        assert e.value.code == gpu_lib.ERR_ARG
    finally:
        del gpu_lib.SCHEDULES["bogus"]
    ctx.free_system(sid)


def test_read_bandwidth_probe(ctx, gpu_lib):
    """The streaming-read reference: a 1 GiB read is bounded above by the datasheet
    8 TB/s and well above a tenth of it; odd sizes, misaligned buffers and reps < 1
    are refused."""
    import torch
    x = torch.ones(1 << 28, dtype=torch.float32, device=ctx.device)       # 1 GiB
    ms = ctx.read_bandwidth(x, 5)
    gbps = x.numel() * 4 / (ms * 1e-3) / 1e9
    print("[gpu] read probe 1 GiB: %.3f ms, %.0f GB/s" % (ms, gbps), flush=True)
    assert 800.0 < gbps < 8000.0
    lib = gpu_lib.lib()
    import ctypes as C
    out = C.c_double()
    p = x.data_ptr()
    for ptr, nbytes, reps in ((p, 24, 1), (p + 4, 1024, 1), (p, 1024, 0), (0, 1024, 1)):
        rc = lib.mqct_read_bandwidth(ctx.h, C.c_void_p(ptr), nbytes, reps, C.byref(out))
        assert rc == gpu_lib.ERR_ARG, (ptr - p, nbytes, reps, rc)
