"""Python access to the FP64 CPU oracle (oracle.cpp).

TEST INFRASTRUCTURE: only the tests, the smoke check and the benchmark's CPU
baseline use this package.  It never imports the GPU library and the GPU
library never imports it; the two share only the seeded inputs from `synth`.
"""
import ctypes as C
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.cpp")
_LIB = os.path.join(_HERE, "liboracle.so")

STATUS = {"EXITED": 1, "MAX_STEPS": 2, "STEP_UNDERFLOW": 4, "BELOW_GRID": 8, "NONFINITE": 16}


def build(force=False):
    """Compile oracle.cpp into liboracle.so with g++ (OpenMP over trajectories)."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["g++", "-O3", "-std=c++17", "-fopenmp", "-fPIC", "-shared",
                               "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


class _Sys(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("R", C.c_void_p), ("E", C.c_void_p),
                ("M", C.c_void_p), ("M2", C.c_void_p), ("dM", C.c_void_p), ("dM2", C.c_void_p),
                ("jx_nnz", C.c_int32), ("jx_row", C.c_void_p), ("jx_col", C.c_void_p),
                ("jx_val", C.c_void_p), ("mu", C.c_double), ("literal_phase", C.c_int32),
                ("plant_coriolis_flip", C.c_int32), ("decoupled", C.c_int32),
                ("drv", C.c_void_p), ("drv2", C.c_void_p)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = C.CDLL(build())
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        _lib.oracle_spline_prepare.argtypes = [i32, vp, i64, vp, vp]
        _lib.oracle_spline_eval.argtypes = [i32, vp, i64, vp, vp, d, vp, vp]
        _lib.oracle_spline_eval.restype = i32
        _lib.oracle_rhs.argtypes = [vp, d, vp, vp]
        _lib.oracle_rhs.restype = d
        _lib.oracle_total_energy.argtypes = [vp, d, vp]
        _lib.oracle_dp5_error.argtypes = [vp, d, vp, d, d, d, vp]
        _lib.oracle_dp5_error.restype = d
        _lib.oracle_total_energy.restype = d
        _lib.oracle_propagate.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, i32, vp, vp,
                                          d, d, i64, d] + [vp] * 10
        _lib.oracle_tangent_rk4.argtypes = [vp, i64, vp, vp, vp, vp, vp, vp, vp, vp]
        _lib.oracle_cross_sections.argtypes = [i64, i32, vp, vp, vp, vp, i32, d, vp]
        _lib.oracle_threads.restype = i32
        _lib.oracle_cg.argtypes = [i32] * 6
        _lib.oracle_cg.restype = d
        _lib.oracle_coupling_angular.argtypes = [i32, vp, vp, vp, vp, i32, vp, vp, i32, i32,
                                                 vp, vp, vp, vp, i32, vp, vp]
        _lib.oracle_coupling_angular.restype = i32
    return _lib


def threads():
    """OpenMP threads the oracle's parallel loops use."""
    return int(lib().oracle_threads())


def _p(a):
    return None if a is None else a.ctypes.data


def _f64(a):
    return None if a is None else np.ascontiguousarray(a, dtype=np.float64)


def spline_prepare(x, y):
    """Natural-spline second derivatives of the columns of y[K, ...] on knots x[K]."""
    x = _f64(x)
    y = _f64(y)
    y2 = np.empty_like(y)
    ncol = int(np.prod(y.shape[1:])) if y.ndim > 1 else 1
    lib().oracle_spline_prepare(len(x), _p(x), ncol, _p(y), _p(y2))
    return y2


def spline_eval(x, y, y2, r):
    x = _f64(x); y = _f64(y); y2 = _f64(y2)
    shape = y.shape[1:]
    ncol = int(np.prod(shape)) if shape else 1
    v = np.empty(ncol); d = np.empty(ncol)
    below = lib().oracle_spline_eval(len(x), _p(x), ncol, _p(y), _p(y2), float(r), _p(v), _p(d))
    return v.reshape(shape), d.reshape(shape), bool(below)


class OracleSystem:
    """A system prepared for the oracle: complex tables and their spline curvature."""

    def __init__(self, system, literal_phase=False, tables=None, tangent_tables=None,
                 plant_coriolis_flip=False, driver=None, knots=None):
        """driver: U(R_k) [K] hartree -- switches to decoupled (AT) dynamics, in
        which the trajectory is driven by the natural spline of U and feels no
        force or torque from the quantum state.

        knots: (R_sub, M_sub, M2_sub) -- only a run of consecutive knots of the
        grid with the tables there and their natural-spline second derivatives of
        the whole grid (see rank_q_knot_tables), for systems too large to hold at
        every knot; trajectories must stay inside that run of knots."""
        self.N = int(system.E.shape[0])
        self.E = _f64(system.E)
        if knots is not None:
            R_sub, M_sub, M2_sub = knots
            self.R = _f64(R_sub)
            self.K = int(self.R.shape[0])
            self.M = np.ascontiguousarray(M_sub, dtype=np.complex128)
            self.M2 = np.ascontiguousarray(M2_sub, dtype=np.complex128).view(np.float64) \
                .reshape(self.K, self.N, self.N, 2)
        else:
            M = system.M if tables is None else tables
            self.K = int(system.R_grid.shape[0])
            self.R = _f64(system.R_grid)
            self.M = np.ascontiguousarray(M, dtype=np.complex128)
            self.M2 = spline_prepare(self.R, self.M.view(np.float64).reshape(self.K, -1)) \
                .reshape(self.K, self.N, self.N, 2)
        self.dM = self.dM2 = None
        if tangent_tables is not None:
            self.dM = np.ascontiguousarray(tangent_tables, dtype=np.complex128)
            self.dM2 = spline_prepare(self.R, self.dM.view(np.float64).reshape(self.K, -1)) \
                .reshape(self.K, self.N, self.N, 2)
        self.jx_row = np.ascontiguousarray(system.jx_row, np.int32)
        self.jx_col = np.ascontiguousarray(system.jx_col, np.int32)
        self.jx_val = _f64(system.jx_val)
        self.mu = float(system.mu)
        self.system = system
        self.drv = self.drv2 = None
        if driver is not None:
            self.drv = _f64(driver).reshape(self.K)
            self.drv2 = spline_prepare(self.R, self.drv.reshape(self.K, 1)).reshape(self.K)
        self.s = _Sys(self.N, self.K, _p(self.R), _p(self.E), _p(self.M), _p(self.M2),
                      _p(self.dM), _p(self.dM2), len(self.jx_val), _p(self.jx_row),
                      _p(self.jx_col), _p(self.jx_val), self.mu, 1 if literal_phase else 0,
                      1 if plant_coriolis_flip else 0, 1 if driver is not None else 0,
                      _p(self.drv), _p(self.drv2))

    def rhs(self, t, y):
        y = _f64(y)
        f = np.empty_like(y)
        eq = lib().oracle_rhs(C.byref(self.s), float(t), _p(y), _p(f))
        return f, eq

    def dp5_error(self, t, y, h, rtol, atol):
        """(error norm, fifth-order solution) of one Dormand-Prince 5(4) attempt of
        size h from (t, y)."""
        y = _f64(y)
        ynew = np.empty_like(y)
        en = lib().oracle_dp5_error(C.byref(self.s), float(t), _p(y), float(h), float(rtol),
                                    float(atol), _p(ynew))
        return en, ynew

    def total_energy(self, t, y):
        y = _f64(y)
        return lib().oracle_total_energy(C.byref(self.s), float(t), _p(y))

    def propagate(self, batch=None, *, init_channel=None, a0=None, classical0=None,
                  E_coll=None, b=None, R0=None, t0=None, method="rk4", dt=None, n_steps=None,
                  rtol=1e-8, atol=1e-8, max_steps=100000, h_min=1e-6):
        if batch is not None:
            init_channel = batch.init_channel if init_channel is None else init_channel
            E_coll = batch.E_coll if E_coll is None else E_coll
            b = batch.b if b is None else b
            R0 = batch.R0 if R0 is None else R0
            dt = batch.dt if dt is None else dt
            n_steps = batch.n_steps if n_steps is None else n_steps
        if classical0 is not None:
            B = int(np.asarray(classical0).reshape(-1, 6).shape[0])
        else:
            B = int(np.asarray(E_coll).shape[0])
        N = self.N
        ic = None if init_channel is None else np.ascontiguousarray(init_channel, np.int32)
        a0c = None if a0 is None else np.ascontiguousarray(
            np.asarray(a0, np.complex128).reshape(B, N)).view(np.float64)
        c0 = _f64(None if classical0 is None else np.reshape(classical0, (B, 6)))
        Ec, bb, r0 = _f64(E_coll), _f64(b), _f64(R0)
        t0c = _f64(t0)
        dtc = _f64(np.broadcast_to(np.asarray(dt if dt is not None else 0.0, np.float64), (B,)))
        ns = np.ascontiguousarray(np.broadcast_to(
            np.asarray(n_steps if n_steps is not None else 0, np.int64), (B,)))
        out = {
            "P": np.empty((B, N)), "a_final": np.empty((B, N), np.complex128),
            "classical": np.empty((B, 6)), "t_final": np.empty(B),
            "steps": np.empty(B, np.int64), "rejects": np.empty(B, np.int64),
            "status": np.empty(B, np.int32), "norm_err": np.empty(B),
            "energy_err": np.empty(B), "angmom_err": np.empty(B)}
        lib().oracle_propagate(
            C.byref(self.s), B, _p(ic), _p(a0c), _p(c0), _p(Ec), _p(bb), _p(r0), _p(t0c),
            0 if method == "rk4" else 1, _p(dtc), _p(ns), float(rtol), float(atol),
            int(max_steps), float(h_min),
            _p(out["P"]), _p(out["a_final"]), _p(out["classical"]), _p(out["t_final"]),
            _p(out["steps"]), _p(out["rejects"]), _p(out["status"]), _p(out["norm_err"]),
            _p(out["energy_err"]), _p(out["angmom_err"]))
        return out

    def tangent_rk4(self, batch):
        assert self.dM is not None, "tangent tables required"
        B, N = batch.B, self.N
        P = np.empty((B, N)); dP = np.empty((B, N))
        ic = np.ascontiguousarray(batch.init_channel, np.int32)
        Ec, bb, r0 = _f64(batch.E_coll), _f64(batch.b), _f64(batch.R0)
        dtc = _f64(batch.dt)
        ns = np.ascontiguousarray(batch.n_steps, np.int64)
        lib().oracle_tangent_rk4(C.byref(self.s), B, _p(ic), _p(Ec), _p(bb), _p(r0), _p(dtc),
                                 _p(ns), _p(P), _p(dP))
        return P, dP


def rank_q_knot_tables(R, phi, v_diag, H, ks, scale=1.0):
    """Tables of the form M(R_k) = scale (sum_q phi[k, q] H_q + v_diag[k] 1) at the
    consecutive knots ks only, with the natural-spline second derivatives of M on
    the whole grid R at those knots.  The spline's second derivatives are linear
    in the tabulated values, so those of M are the factors' (each column phi[:, q]
    and v_diag splined on the whole grid) combined in the same way -- the same
    numbers, up to rounding, as splining every element of M.  Returns (R[ks],
    M [len(ks), N, N], M2 [len(ks), N, N])."""
    ks = np.asarray(ks)
    assert np.all(np.diff(ks) == 1), "a run of consecutive knots"
    R = _f64(R)
    phi = _f64(phi)
    v_diag = _f64(v_diag)
    phi2 = spline_prepare(R, phi)
    v2 = spline_prepare(R, v_diag.reshape(-1, 1)).reshape(-1)
    Q, N, _ = H.shape
    Hf = np.ascontiguousarray(H).view(np.float64).reshape(Q, 2 * N * N)
    eye = np.arange(N)

    def at(coef, diag):
        out = (coef @ Hf).view(np.complex128).reshape(-1, N, N)
        for i in range(out.shape[0]):
            out[i] = 0.5 * (out[i] + out[i].conj().T)
            out[i][eye, eye] += diag[i]
            out[i] *= scale
        return out

    return R[ks], at(phi[ks], v_diag[ks]), at(phi2[ks], v2[ks])


def cross_sections(init_level, b, P, level_of_channel, n_levels, b_max):
    P = _f64(P)
    B, N = P.shape
    sig = np.empty((n_levels, n_levels))
    il = np.ascontiguousarray(init_level, np.int32)
    lc = np.ascontiguousarray(level_of_channel, np.int32)
    bb = _f64(b)
    lib().oracle_cross_sections(B, N, _p(il), _p(bb), _p(P), _p(lc), int(n_levels),
                                float(b_max), _p(sig))
    return sig


# ---------------------------------------------------------------------------
# coupling matrix of an asymmetric top + linear rotor (Section II, Eq. 17)

def cg(j1, m1, j2, m2, J, M):
    """Clebsch-Gordan coefficient <j1 m1 j2 m2 | J M> (Racah's closed form)."""
    return float(lib().oracle_cg(j1, m1, j2, m2, J, M))


def coupling_angular(basis, lam1, mu1, lam2, lam, rows=None):
    """G[t, n'', n']: Eq. 17 with v_t = 1 for each term t = (lam1, mu1, lam2, lam).

    basis: channels (j, m, rot1, j2) and rotor-1 states (rot1_j, b) as built by
    synth.coupling.top_rotor_basis.  rows: only these final states n'' (the
    result is then G[t, q, n'] for n'' = rows[q])."""
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    j, m, r1, j2 = i32(basis.j), i32(basis.m), i32(basis.rot1), i32(basis.j2)
    rj, b = i32(basis.rot1_j), _f64(basis.b)
    l1, u1, l2, l = i32(lam1), i32(mu1), i32(lam2), i32(lam)
    N, T = j.shape[0], l1.shape[0]
    rr = None if rows is None else i32(rows)
    nr = N if rr is None else rr.shape[0]
    G = np.empty((T, nr, N))
    rc = lib().oracle_coupling_angular(N, _p(j), _p(m), _p(r1), _p(j2), rj.shape[0], _p(rj),
                                       _p(b), b.shape[1], T, _p(l1), _p(u1), _p(l2), _p(l),
                                       nr, _p(rr), _p(G))
    if rc != 0:
        raise ValueError("coupling_angular: index or b layout out of range")
    return G


def coupling_tables(basis, expansion, rows=None):
    """M[k, n'', n'] = sum_t v_t(R_k) G_t (Eq. 12 into Eq. 17), and the G_t."""
    G = coupling_angular(basis, expansion.lam1, expansion.mu1, expansion.lam2, expansion.lam,
                         rows=rows)
    M = np.einsum("tk,tab->kab", np.asarray(expansion.v, np.float64), G)
    return M, G
