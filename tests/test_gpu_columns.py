"""GPU parity of coordinate-list (truncated) coupling tables on the columns
schedule: decoupled (AT) dynamics of many initial states per classical path
(Section III: AT-MQCT, the trajectories carried 100 initial states; the coupling
matrices kept only the elements above a threshold).

* The structural nonzeros of the two-rotor tables (N = 256, real, 91 % zeros) as a
  shuffled coordinate list; three paths of 5, 1 and 130 columns (the last split
  into groups of 128 and 2); FP64 tables within 1e-9 of the oracle per channel,
  FP32 within 1e-4; against the dense tables' AT on the per-trajectory schedule.
* Complex Hermitian tables (asymmetric top + atom, N = 84) truncated to the
  elements above a threshold at some knot, as the paper's matrices were (its
  1 cm^-1; here 16.7 cm^-1, which keeps the largest 30 % of the synthetic
  elements): the oracle on the same truncated tables, initial amplitudes given
  as vectors.
* A screened coupling build (top + rotor, N = 504, Eq. 17, with J_x): the
  builder's device output loaded as it is.
* Errors: a missing (m, n) partner, a repeated element, an index out of range,
  unequal partners, a non-finite value; batches the schedule does not run.
"""
import sys

import numpy as np
import pytest

import oracle
from synth import coupling as CP
from synth import systems as S
from synth import units as U

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


def driver_of(M):
    """The average diagonal of the tables: an isotropic driving potential."""
    return np.real(np.einsum("knn->k", M)) / M.shape[1]


def coo_of(M, drop=0.0, seed=0):
    """The elements whose magnitude exceeds `drop` at some knot, in (n, m) or (m, n),
    as a shuffled coordinate list (rows, cols, values [K, n])."""
    A = np.abs(M).max(axis=0)
    keep = (A > drop) | (A.T > drop)
    rows, cols = np.nonzero(keep)
    p = np.random.default_rng(seed).permutation(rows.shape[0])
    rows, cols = rows[p], cols[p]
    return rows.astype(np.int32), cols.astype(np.int32), np.ascontiguousarray(M[:, rows, cols]), keep


def truncated(s, keep):
    """The system with the dropped elements set to zero at every knot."""
    t = S.System(**{k: getattr(s, k) for k in s.__dataclass_fields__})
    t.M = np.where(keep[None, :, :], s.M, 0.0)
    return t


def paths_batch(s, sizes, rng, n_steps, dt, U_cm, b_max_ang, R0_bohr):
    """len(sizes) paths (each its own E_coll, b, R0), sizes[i] columns on path i with
    initial channels 0, 1, ..."""
    parts = []
    for i, n in enumerate(sizes):
        one = S.mc_batch(s, 1, U_cm[i], b_max_ang, [0], rng, n_steps=n_steps, dt=dt,
                         R0_bohr=R0_bohr[i])
        idx = np.zeros(n, np.int64)
        sub = one.subset(idx)
        sub.init_channel[:] = np.arange(n) % s.N
        parts.append(sub)
    out = parts[0]
    for p in parts[1:]:
        out = S.Batch(*[np.concatenate([getattr(out, f), getattr(p, f)]) if isinstance(
            getattr(out, f), np.ndarray) else getattr(out, f) for f in S.Batch.__dataclass_fields__])
    return out


def run_columns(ctx, sid, N, b, **kw):
    g = ctx.run_host([sid] * b.B, [N] * b.B, schedule="columns", dynamics="at",
                     init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0, dt=b.dt,
                     n_steps=b.n_steps, **kw)
    g["P"] = g["P"].reshape(b.B, N)
    return g


@pytest.fixture(scope="module")
def rotor_rotor():
    (s,), _ = S.config4(n_traj=1, n_steps=1)                     # N = 256, real
    rng = np.random.default_rng(41)
    R0 = [s.R_grid[50], s.R_grid[45], s.R_grid[55]]          # 11.5-13.2 bohr, inside the coupling
    b = paths_batch(s, [5, 1, 130], rng, 300, 15.0, [400.0, 900.0, 250.0], 2.0, R0)
    return s, b


@pytest.mark.parametrize("storage", ["R64", "R32"])
def test_columns_two_rotor_structural_nonzeros(ctx, rotor_rotor, storage):
    s, b = rotor_rotor
    rows, cols, vals, keep = coo_of(s.M)
    Udrv = driver_of(s.M)
    say("columns N=%d %s: %d of %d elements, paths of 5, 1 and 130 columns x %d steps" % (
        s.N, storage, rows.shape[0], s.N * s.N, b.n_steps[0]))
    sid = ctx.load_system_coo(R_grid=s.R_grid, E=s.E, rows=rows, cols=cols, values=vals, mu=s.mu,
                              jx=(s.jx_row, s.jx_col, s.jx_val), storage=storage)
    assert ctx.system_bytes(sid) == 2 * s.K * rows.shape[0] * (8 if storage == "R64" else 4)
    ctx.set_driver(sid, Udrv)
    g = run_columns(ctx, sid, s.N, b)
    ctx.free_system(sid)
    pick = [0, 3, 4, 5, 6, 100, 133, 134, 135]         # the last two sit in the second group
    o = oracle.OracleSystem(s, driver=Udrv).propagate(b.subset(pick))
    d = np.max(np.abs(g["P"][pick] - o["P"]))
    dc = np.max(np.abs(g["classical"][pick] - o["classical"]) / (1 + np.abs(o["classical"])))
    say("  max|dP| %.3e, classical %.3e, max|norm-1| %.2e" % (d, dc, np.max(np.abs(g["norm_err"]))))
    moved = 1.0 - o["P"][np.arange(len(pick)), b.init_channel[pick]]
    say("  population leaving the initial channel: %.2e .. %.2e" % (moved.min(), moved.max()))
    assert moved.max() > 1e-2
    assert d < (1e-9 if storage == "R64" else 1e-4)
    assert dc < 1e-10
    assert np.max(np.abs(g["energy_err"][pick] - o["energy_err"])) < 1e-10
    assert np.all(g["angmom_err"] == 0.0)
    assert np.array_equal(g["steps"], b.n_steps) and np.array_equal(g["status"][pick], o["status"])
    # columns of one path share it exactly
    for lo, hi in ((0, 5), (6, 136)):
        assert np.all(g["classical"][lo:hi] == g["classical"][lo])
    if storage == "R64":
        dense = ctx.load_system(s)
        ctx.set_driver(dense, Udrv)
        gg = ctx.run_host([dense] * b.B, [s.N] * b.B, schedule="gemv", dynamics="at",
                          init_channel=b.init_channel, E_coll=b.E_coll, b=b.b, R0=b.R0,
                          dt=b.dt, n_steps=b.n_steps)
        ctx.free_system(dense)
        dd = np.max(np.abs(gg["P"].reshape(b.B, s.N) - g["P"]))
        say("  against the dense tables on the per-trajectory schedule: %.3e" % dd)
        assert dd < 1e-12


@pytest.mark.parametrize("storage", ["C128", "C64"])
def test_columns_complex_truncated_at_one_wavenumber(ctx, storage):
    (s,), _ = S.config2(n_traj=1, jmax=3)                          # N = 84, complex
    drop = np.percentile(np.abs(s.M).max(axis=0), 70)               # 16.7 cm^-1
    rows, cols, vals, keep = coo_of(s.M, drop=drop, seed=3)
    assert rows.shape[0] < 0.5 * s.N * s.N
    st = truncated(s, keep)
    Udrv = driver_of(st.M)
    rng = np.random.default_rng(43)
    b = paths_batch(s, [3, 2], rng, 400, 12.0, [700.0, 300.0], 2.0, [14.0, 12.5])
    a0 = rng.standard_normal((b.B, s.N)) + 1j * rng.standard_normal((b.B, s.N))
    a0 /= np.linalg.norm(a0, axis=1, keepdims=True)
    say("columns N=%d %s: %d of %d elements above %.3g cm^-1, a0 vectors" % (
        s.N, storage, rows.shape[0], s.N * s.N, drop / U.cm_to_hartree(1.0)))
    sid = ctx.load_system_coo(R_grid=s.R_grid, E=s.E, rows=rows, cols=cols, values=vals, mu=s.mu,
                              jx=(s.jx_row, s.jx_col, s.jx_val), storage=storage)
    ctx.set_driver(sid, Udrv)
    g = run_columns(ctx, sid, s.N, b, a0=a0.reshape(-1))
    ctx.free_system(sid)
    o = oracle.OracleSystem(st, driver=Udrv).propagate(b, a0=a0)
    d = np.max(np.abs(g["P"] - o["P"]))
    da = np.max(np.abs(g["a_final"].reshape(b.B, s.N) - o["a_final"]))
    say("  max|dP| %.3e, max|da| %.3e" % (d, da))
    assert d < (1e-9 if storage == "C128" else 1e-4)
    assert np.max(np.abs(g["norm_err"] - o["norm_err"])) < (1e-10 if storage == "C128" else 1e-5)


def test_columns_screened_builder_output(ctx):
    """The builder's screened output (device arrays, any order) loaded directly."""
    basis = CP.top_rotor_basis(3, (0, 2), order="m")              # N = 504
    terms = CP.select_terms(CP.expansion_terms(), 40, seed=1)
    Rg = CP.log_grid(63)
    ex = CP.synthetic_expansion(terms, Rg, seed=1)
    vs = CP.synthetic_expansion(terms, np.array(CP.PAPER_SCREEN_R), seed=1).v
    thr = U.cm_to_hartree(0.05)
    out = ctx.build_couplings_sparse(basis, ex, vs, thr)
    n = out["n_kept"]
    dense = ctx.build_couplings(basis, ex)["M"].cpu().numpy()
    r, c = out["rows"].cpu().numpy(), out["cols"].cpu().numpy()
    keep = np.zeros((basis.N, basis.N), bool)
    keep[r, c] = True
    s = CP.system_from_tables(basis, Rg, np.where(keep[None], dense, 0.0))
    Udrv = driver_of(s.M)
    say("columns screened build N=%d: %d kept of %d" % (basis.N, n, basis.N ** 2))
    sid = ctx.load_system_coo(R_grid=Rg, E=basis.E, rows=out["rows"], cols=out["cols"],
                              values=out["values"], mu=s.mu,
                              jx=(basis.jx_row, basis.jx_col, basis.jx_val))
    ctx.set_driver(sid, Udrv)
    rng = np.random.default_rng(44)
    b = paths_batch(s, [4, 3], rng, 250, 15.0, [150.0, 600.0], 2.0, [14.0, 16.0])
    g = run_columns(ctx, sid, basis.N, b)
    ctx.free_system(sid)
    o = oracle.OracleSystem(s, driver=Udrv).propagate(b)
    d = np.max(np.abs(g["P"] - o["P"]))
    say("  max|dP| %.3e, P off the initial channel up to %.2e" % (
        d, np.max(1.0 - g["P"][np.arange(b.B), b.init_channel])))
    assert d < 1e-9
    assert np.array_equal(g["status"], o["status"])


def test_columns_errors(ctx, gpu_lib):
    (s,), _ = S.config1(n_traj=1, n_steps=1, jmax=2)               # N = 9, real
    rows, cols, vals, keep = coo_of(s.M)
    kw = dict(R_grid=s.R_grid, E=s.E, mu=s.mu)
    # option values out of range
    for name, v in (("col_workspace", -1), ("per_launch", 0), ("per_launch", 65)):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.set_option(name, v)
        assert e.value.code == -1, (name, v)

    def refused(code, r, c, v):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.load_system_coo(rows=r, cols=c, values=v, **kw)
        assert e.value.code == code, e.value

    off = np.where(rows != cols)[0][0]
    drop = np.ones(rows.shape[0], bool)
    drop[off] = False
    refused(gpu_lib.ERR_ARG, rows[drop], cols[drop], np.ascontiguousarray(vals[:, drop]))
    refused(gpu_lib.ERR_ARG, np.append(rows, rows[0]), np.append(cols, cols[0]),
            np.ascontiguousarray(np.concatenate([vals, vals[:, :1]], axis=1)))
    bad = rows.copy()
    bad[1] = s.N
    refused(gpu_lib.ERR_ARG, bad, cols, vals)
    v2 = vals.copy()
    v2[:, off] += 1e-6 * np.abs(vals).max()
    refused(gpu_lib.ERR_NOT_HERMITIAN, rows, cols, v2)
    v3 = vals.copy()
    v3[7, 2] = np.nan
    refused(gpu_lib.ERR_NONFINITE, rows, cols, v3)
    sid = ctx.load_system_coo(rows=rows, cols=cols, values=vals, **kw)
    dense = ctx.load_system(s)
    common = dict(init_channel=[0], E_coll=[U.cm_to_hartree(500.0)], b=[1.0], dt=[10.0],
                  n_steps=[5])
    cases = [(sid, dict(dynamics="at")),                                    # no driver yet
             (sid, dict(dynamics="ehrenfest", schedule="columns")),
             (sid, dict(dynamics="at", schedule="gemv")),
             (sid, dict(dynamics="at", schedule="binned")),
             (dense, dict(dynamics="at", schedule="columns"))]
    codes = [gpu_lib.ERR_STATE] + [gpu_lib.ERR_UNSUPPORTED] * 4
    for (x, extra), code in zip(cases, codes):
        with pytest.raises(gpu_lib.MQCTError) as e:
            ctx.run_host([x], [s.N], **common, **extra)
        assert e.value.code == code, (extra, e.value)
    ctx.set_driver(sid, driver_of(s.M))
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.run_host([sid], [s.N], integrator="dp5", dynamics="at", init_channel=[0],
                     E_coll=common["E_coll"], b=[1.0])
    assert e.value.code == gpu_lib.ERR_UNSUPPORTED
    with pytest.raises(gpu_lib.MQCTError) as e:
        ctx.set_params(sid, np.ones((1, s.K)), np.zeros(1, np.int32), np.eye(s.N)[None])
    assert e.value.code == gpu_lib.ERR_UNSUPPORTED
    g = ctx.run_host([sid], [s.N], dynamics="at", **common)
    assert g["status"][0] == 0 and abs(g["norm_err"][0]) < 1e-12
    ctx.free_system(sid)
    ctx.free_system(dense)


def test_columns_paper_size_properties(ctx):
    """The paper's size: the 206,350-state p-H2O + p-H2 basis and its screened
    matrices (13 M kept elements, FP64 tables), one path in the interaction region
    carrying four columns: e_i, e_j, (e_i + e_j)/sqrt 2 and (e_i - i e_j)/sqrt 2.  The
    oracle cannot hold this basis; the properties that hold at any size are checked
    instead: the quantum equations are linear in the amplitudes along a fixed path
    (AT), so the third and fourth columns equal those combinations of the first two;
    the propagation is unitary (norm); every column follows the same path."""
    basis = CP.para_h2o_para_h2_basis()
    terms = CP.select_terms(CP.expansion_terms(), 83, seed=0)
    Rg = CP.log_grid(63)
    ex = CP.synthetic_expansion(terms, Rg, seed=0)
    vs = CP.synthetic_expansion(terms, np.array(CP.PAPER_SCREEN_R), seed=0).v
    out = ctx.build_couplings_sparse(basis, ex, vs, U.cm_to_hartree(CP.PAPER_SCALE_DROP_CM))
    say("paper size: N=%d, %d kept elements" % (basis.N, out["n_kept"]))
    sid = ctx.load_system_coo(R_grid=Rg, E=basis.E, rows=out["rows"], cols=out["cols"],
                              values=out["values"], mu=U.amu_to_me(1.8),
                              jx=(basis.jx_row, basis.jx_col, basis.jx_val))
    del out
    iso = [t for t, tm in enumerate(terms) if tuple(tm) == (0, 0, 0, 0)][0]
    ctx.set_driver(sid, ex.v[iso] / (2.0 * np.pi))
    i, j = 0, int(np.argsort(basis.E, kind="stable")[37])
    N, B = basis.N, 4
    a0 = np.zeros((B, N), np.complex128)
    a0[0, i] = 1.0
    a0[1, j] = 1.0
    a0[2, i] = a0[2, j] = 1.0 / np.sqrt(2.0)
    a0[3, i], a0[3, j] = 1.0 / np.sqrt(2.0), -1j / np.sqrt(2.0)
    g = ctx.run_host([sid] * B, [N] * B, schedule="columns", dynamics="at", a0=a0.reshape(-1),
                     E_coll=np.full(B, U.cm_to_hartree(300.0)), b=np.full(B, 2.0),
                     R0=np.full(B, 7.0), dt=np.full(B, 10.0), n_steps=np.full(B, 40))
    ctx.free_system(sid)
    a = g["a_final"].reshape(B, N)
    lin = max(np.max(np.abs(a[2] - (a[0] + a[1]) / np.sqrt(2.0))),
              np.max(np.abs(a[3] - (a[0] - 1j * a[1]) / np.sqrt(2.0))))
    say("  linearity %.2e, max|norm-1| %.2e, population off the start: %.2e, %.2e" % (
        lin, np.max(np.abs(g["norm_err"])), 1 - abs(a[0, i]) ** 2, 1 - abs(a[1, j]) ** 2))
    assert 1 - abs(a[0, i]) ** 2 > 1e-6
    assert lin < 1e-12
    assert np.max(np.abs(g["norm_err"])) < 1e-12
    assert np.all(g["classical"] == g["classical"][0]) and np.all(g["status"] == 0)


def test_columns_ragged_steps_start_states_and_t0(ctx):
    """Groups of different lengths in one call (0, 3 and 10 RK4 steps: a group that
    stops early keeps its amplitudes while the others go on), and a path given by
    its start state (classical0) at t0 != 0 (the phases e^{-iE t} start there),
    against the oracle; every column of a path on the same path bit for bit."""
    (s,), _ = S.config1(n_traj=1, n_steps=1, jmax=3)               # N = 16, real
    rows, cols, vals, keep = coo_of(s.M, seed=9)
    Udrv = driver_of(s.M)
    sid = ctx.load_system_coo(R_grid=s.R_grid, E=s.E, rows=rows, cols=cols, values=vals, mu=s.mu,
                              jx=(s.jx_row, s.jx_col, s.jx_val))
    ctx.set_driver(sid, Udrv)
    rng = np.random.default_rng(47)
    b = paths_batch(s, [2, 3, 2], rng, 10, 25.0, [500.0, 500.0, 800.0], 2.0,
                    [s.R_grid[60], s.R_grid[60], s.R_grid[70]])
    b.n_steps[:] = [0, 0, 3, 3, 3, 10, 10]
    g = run_columns(ctx, sid, s.N, b)
    o = oracle.OracleSystem(s, driver=Udrv).propagate(b)
    d = np.max(np.abs(g["P"] - o["P"]))
    say("ragged columns N=%d: steps %s, max|dP| %.3e" % (s.N, g["steps"].tolist(), d))
    assert d < 1e-12 and np.array_equal(g["steps"], b.n_steps)
    assert np.all(g["P"][[0, 1], b.init_channel[[0, 1]]] == 1.0)
    assert np.max(np.abs(g["t_final"] - o["t_final"])) == 0.0
    # a start state and t0
    c0 = np.array([[14.0, 0.5 * np.pi, 0.3, -2.0, 0.0, 9.0]] * 3)
    t0 = np.full(3, 123.5)
    ic = np.array([1, 4, 7], np.int32)
    g = ctx.run_host([sid] * 3, [s.N] * 3, schedule="columns", dynamics="at", init_channel=ic,
                     classical0=c0.reshape(-1), t0=t0, dt=np.full(3, 20.0),
                     n_steps=np.full(3, 60))
    o = oracle.OracleSystem(s, driver=Udrv).propagate(init_channel=ic, classical0=c0, t0=t0,
                                                      dt=np.full(3, 20.0), n_steps=np.full(3, 60))
    d = np.max(np.abs(g["P"].reshape(3, s.N) - o["P"]))
    dc = np.max(np.abs(g["classical"] - o["classical"]) / (1 + np.abs(o["classical"])))
    say("  classical0 at t0 = 123.5: max|dP| %.3e, classical %.3e" % (d, dc))
    assert d < 1e-12 and dc < 1e-12
    assert np.all(g["classical"] == g["classical"][0])
    assert np.max(np.abs(g["t_final"] - o["t_final"])) < 1e-12 * np.max(o["t_final"])
    ctx.free_system(sid)


def test_columns_workspace_cap_runs_in_passes(ctx, gpu_lib, rotor_rotor):
    """A workspace cap below the whole batch's need: the path groups (5, 1, 128 and
    2 columns, 4 x 300 RK4 steps, N = 256) run in passes of one or two groups, with
    the results of the single pass bit for bit; a cap below one group's need is an
    allocation error, and the library stays usable."""
    s, b = rotor_rotor
    rows, cols, vals, keep = coo_of(s.M)
    sid = ctx.load_system_coo(R_grid=s.R_grid, E=s.E, rows=rows, cols=cols, values=vals, mu=s.mu,
                              jx=(s.jx_row, s.jx_col, s.jx_val), storage="R32")
    ctx.set_driver(sid, driver_of(s.M))
    one_group = s.N * 128 * 80                  # columns of one group, FP32 tables
    try:
        ref = run_columns(ctx, sid, s.N, b)
        for cap in (int(1.2 * one_group), int(2.2 * one_group)):
            ctx.set_option("col_workspace", cap)
            g = run_columns(ctx, sid, s.N, b)
            say("columns workspace cap %.1f MB: max|dP| against one pass %.1e" % (
                cap / 1e6, np.max(np.abs(g["P"] - ref["P"]))))
            for k in ("P", "classical", "norm_err", "energy_err", "status", "steps", "t_final"):
                assert np.array_equal(g[k], ref[k]), k
        ctx.set_option("col_workspace", one_group // 2)
        with pytest.raises(gpu_lib.MQCTError) as ei:
            run_columns(ctx, sid, s.N, b)
        assert ei.value.code == -4 and "columns workspace" in str(ei.value)
    finally:
        ctx.set_option("col_workspace", 0)
    g = run_columns(ctx, sid, s.N, b)
    assert np.array_equal(g["P"], ref["P"])
    ctx.free_system(sid)
