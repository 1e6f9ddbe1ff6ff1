"""MI355X (gfx950) batched Ehrenfest mean-field trajectory propagation (MQCT).

A thin ctypes binding of libmqct (include/mqct.h): argument marshalling only,
every step of the propagation runs in the library's HIP kernels.  PyTorch
provides device memory and the stream.  The binding fails loudly when the
library has not been built or no GPU is visible.

    ctx = Context()                       # on torch's current stream of cuda:0
    sid = ctx.load_system(system, storage="C128")
    out = ctx.run([sid] * B, init_channel=..., E_coll=..., b=..., dt=..., n_steps=...)
    torch.cuda.synchronize(); out["P"]     # final |a_n|^2, concatenated per trajectory
"""
import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmqct.so")

OK, ERR_ARG, ERR_NONFINITE, ERR_NOT_HERMITIAN, ERR_OOM, ERR_DEVICE, ERR_UNSUPPORTED, ERR_STATE = \
    0, -1, -2, -3, -4, -5, -6, -7
DTYPES = {"R64": 0, "C128": 1, "R32": 2, "C64": 3}
INTEGRATORS = {"rk4": 0, "dp5": 1}
DYNAMICS = {"ehrenfest": 0, "at": 1}
LAYOUTS = {"dense": 0, "sparse": 1}
SCHEDULES = {"auto": 0, "gemv": 1, "binned": 2, "queue": 3, "columns": 4}
OPTIONS = {"graphs": 1, "autotune": 2, "chunk": 3, "reset_tuning": 4, "tail": 5, "col_workspace": 6, "per_launch": 7}
MEM_HOST, MEM_DEVICE = 0, 1
STATUS = {"EXITED": 1, "MAX_STEPS": 2, "STEP_UNDERFLOW": 4, "BELOW_GRID": 8, "NONFINITE": 16}

# exported C functions, as declared in include/mqct.h
EXPORTS = ["mqct_create", "mqct_destroy", "mqct_last_error", "mqct_synchronize",
           "mqct_system_load", "mqct_system_bytes", "mqct_system_free", "mqct_run",
           "mqct_cross_sections", "mqct_set_profiling", "mqct_profile_read",
           "mqct_system_set_params", "mqct_system_set_theta", "mqct_adjoint",
           "mqct_set_option", "mqct_tuning_report", "mqct_system_set_driver",
           "mqct_coupling_build", "mqct_xs_symmetrize", "mqct_rate_coefficients",
           "mqct_coupling_build_sparse", "mqct_get_state", "mqct_set_state",
           "mqct_state_count", "mqct_run_noalloc", "mqct_read_bandwidth",
           "mqct_system_load_coo"]


class CouplingDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("j", C.c_void_p), ("m", C.c_void_p), ("rot1", C.c_void_p),
                ("j2", C.c_void_p), ("n_rot1", C.c_int32), ("rot1_j", C.c_void_p),
                ("b", C.c_void_p), ("b_stride", C.c_int32), ("T", C.c_int32),
                ("lam1", C.c_void_p), ("mu1", C.c_void_p), ("lam2", C.c_void_p),
                ("lam", C.c_void_p), ("K", C.c_int32), ("v", C.c_void_p)]


class MQCTError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("mqct error %d: %s" % (code, msg))
        self.code = code


class SystemDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("R_grid", C.c_void_p), ("E", C.c_void_p),
                ("in_dtype", C.c_int32), ("M_mem", C.c_int32), ("M", C.c_void_p),
                ("storage", C.c_int32), ("jx_nnz", C.c_int32), ("jx_row", C.c_void_p),
                ("jx_col", C.c_void_p), ("jx_val", C.c_void_p), ("mu", C.c_double),
                ("layout", C.c_int32), ("drop_below", C.c_double)]


class CooDesc(C.Structure):
    _fields_ = [("N", C.c_int32), ("K", C.c_int32), ("R_grid", C.c_void_p), ("E", C.c_void_p),
                ("mu", C.c_double), ("in_dtype", C.c_int32), ("mem", C.c_int32),
                ("n_el", C.c_int64), ("rows", C.c_void_p), ("cols", C.c_void_p),
                ("values", C.c_void_p), ("ld", C.c_int64), ("storage", C.c_int32),
                ("jx_nnz", C.c_int32), ("jx_row", C.c_void_p), ("jx_col", C.c_void_p),
                ("jx_val", C.c_void_p)]


class BatchDesc(C.Structure):
    _fields_ = [("B", C.c_int64), ("system_id", C.c_void_p), ("init_channel", C.c_void_p),
                ("a0", C.c_void_p), ("classical0", C.c_void_p), ("E_coll", C.c_void_p),
                ("b", C.c_void_p), ("R0", C.c_void_p), ("t0", C.c_void_p),
                ("integrator", C.c_int32), ("dt", C.c_void_p), ("n_steps", C.c_void_p),
                ("rtol", C.c_double), ("atol", C.c_double), ("max_steps", C.c_int64),
                ("h_min", C.c_double), ("schedule", C.c_int32), ("dynamics", C.c_int32),
                ("resume", C.c_int32)]


class TrajState(C.Structure):
    """mqct_traj_state: the stored state of one trajectory."""
    _fields_ = [("t", C.c_double), ("t_origin", C.c_double), ("h", C.c_double),
                ("classical", C.c_double * 6), ("E0", C.c_double), ("J0", C.c_double),
                ("R_exit", C.c_double), ("n_origin", C.c_int64), ("steps", C.c_int64),
                ("rejects", C.c_int64), ("attempts", C.c_int64), ("status", C.c_int32),
                ("flags", C.c_int32), ("system_id", C.c_int32), ("N", C.c_int32)]


# the same record as a numpy structured type (host copies of the store)
STATE_DTYPE = np.dtype([("t", "<f8"), ("t_origin", "<f8"), ("h", "<f8"), ("classical", "<f8", (6,)),
                        ("E0", "<f8"), ("J0", "<f8"), ("R_exit", "<f8"), ("n_origin", "<i8"),
                        ("steps", "<i8"), ("rejects", "<i8"), ("attempts", "<i8"),
                        ("status", "<i4"), ("flags", "<i4"), ("system_id", "<i4"), ("N", "<i4")])


class BatchResult(C.Structure):
    _fields_ = [("mem", C.c_int32), ("P", C.c_void_p), ("a_final", C.c_void_p),
                ("classical", C.c_void_p), ("t_final", C.c_void_p), ("steps", C.c_void_p),
                ("rejects", C.c_void_p), ("status", C.c_void_p), ("norm_err", C.c_void_p),
                ("energy_err", C.c_void_p), ("angmom_err", C.c_void_p)]


_lib = None


def lib():
    """The loaded libmqct; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libmqct.so is not built (run __graft_entry__.build())")
        L = C.CDLL(LIB_PATH)
        vp, i32, i64, d = C.c_void_p, C.c_int32, C.c_int64, C.c_double
        L.mqct_create.argtypes = [i32, vp, C.POINTER(vp)]
        L.mqct_create.restype = i32
        L.mqct_destroy.argtypes = [vp]
        L.mqct_destroy.restype = None
        L.mqct_last_error.argtypes = [vp]
        L.mqct_last_error.restype = C.c_char_p
        L.mqct_synchronize.argtypes = [vp]
        L.mqct_synchronize.restype = i32
        L.mqct_system_load.argtypes = [vp, C.POINTER(SystemDesc), C.POINTER(i32)]
        L.mqct_system_load.restype = i32
        L.mqct_system_bytes.argtypes = [vp, i32, C.POINTER(i64)]
        L.mqct_system_bytes.restype = i32
        L.mqct_system_free.argtypes = [vp, i32]
        L.mqct_system_free.restype = i32
        L.mqct_run.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(BatchResult)]
        L.mqct_run.restype = i32
        L.mqct_cross_sections.argtypes = [vp, i32, i64, i32, vp, vp, vp, vp, i32, d, vp]
        L.mqct_cross_sections.restype = i32
        L.mqct_set_profiling.argtypes = [vp, i32]
        L.mqct_set_profiling.restype = i32
        L.mqct_profile_read.argtypes = [vp, C.POINTER(d), C.POINTER(i64), C.POINTER(d)]
        L.mqct_profile_read.restype = i32
        L.mqct_system_load_coo.argtypes = [vp, C.POINTER(CooDesc), C.POINTER(i32)]
        L.mqct_system_load_coo.restype = i32
        L.mqct_read_bandwidth.argtypes = [vp, vp, i64, i32, C.POINTER(d)]
        L.mqct_read_bandwidth.restype = i32
        L.mqct_system_set_params.argtypes = [vp, i32, i32, vp, vp, i32, vp]
        L.mqct_system_set_params.restype = i32
        L.mqct_system_set_theta.argtypes = [vp, i32, vp]
        L.mqct_system_set_theta.restype = i32
        L.mqct_adjoint.argtypes = [vp, C.POINTER(BatchDesc), i32, vp, vp, vp]
        L.mqct_adjoint.restype = i32
        L.mqct_system_set_driver.argtypes = [vp, i32, vp]
        L.mqct_system_set_driver.restype = i32
        L.mqct_set_option.argtypes = [vp, i32, i64]
        L.mqct_set_option.restype = i32
        L.mqct_tuning_report.argtypes = [vp]
        L.mqct_tuning_report.restype = C.c_char_p
        L.mqct_coupling_build.argtypes = [vp, C.POINTER(CouplingDesc), vp, vp]
        L.mqct_coupling_build.restype = i32
        L.mqct_coupling_build_sparse.argtypes = [vp, C.POINTER(CouplingDesc), i32, vp, d, i64,
                                                 vp, vp, vp, C.POINTER(i64)]
        L.mqct_coupling_build_sparse.restype = i32
        L.mqct_xs_symmetrize.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp]
        L.mqct_xs_symmetrize.restype = i32
        L.mqct_rate_coefficients.argtypes = [vp, i32, i32, i32, vp, vp, vp, vp, d, i32, vp, vp]
        L.mqct_rate_coefficients.restype = i32
        L.mqct_get_state.argtypes = [vp, i64, i64, vp, vp]
        L.mqct_get_state.restype = i32
        L.mqct_set_state.argtypes = [vp, i64, i64, vp, vp]
        L.mqct_set_state.restype = i32
        L.mqct_state_count.argtypes = [vp, C.POINTER(i64)]
        L.mqct_state_count.restype = i32
        L.mqct_run_noalloc.argtypes = [vp, C.POINTER(BatchDesc), C.POINTER(BatchResult)]
        L.mqct_run_noalloc.restype = i32
        _lib = L
    return _lib


def _ptr(a):
    if a is None:
        return None
    if hasattr(a, "data_ptr"):
        return a.data_ptr()
    return a.ctypes.data


def _host(a, dtype):
    return None if a is None else np.ascontiguousarray(np.asarray(a), dtype=dtype)


class Context:
    """A library context on one GPU, bound to torch's current stream there."""

    def __init__(self, device=0, stream=None):
        import torch
        if not torch.cuda.is_available():
            raise RuntimeError("no GPU visible: the MQCT propagator runs only on the GPU")
        self.torch = torch
        self.device = torch.device("cuda", device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        h = C.c_void_p()
        code = lib().mqct_create(device, C.c_void_p(stream.cuda_stream), C.byref(h))
        if code != OK:
            raise MQCTError(code, "mqct_create failed")
        self.h = h
        self._keep = []

    def close(self):
        if getattr(self, "h", None):
            lib().mqct_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, code):
        if code != OK:
            raise MQCTError(code, lib().mqct_last_error(self.h).decode())

    def synchronize(self):
        self._check(lib().mqct_synchronize(self.h))

    # ------------------------------------------------------------------ systems
    def load_system(self, system=None, *, R_grid=None, E=None, M=None, jx=None, mu=None,
                    storage=None, layout="dense", drop_below=0.0):
        """Upload a system (tables copied; spline prepared on the device).

        `system` may be any object with R_grid, E, M, jx_row, jx_col, jx_val and mu
        (atomic units).  M may be a numpy array (host) or a CUDA tensor (device),
        real or complex, shaped [K, N, N].  storage: "R64", "C128", "R32", "C64"
        (default: the input's own precision).  layout="sparse" keeps only the
        elements whose magnitude exceeds drop_below (hartree) at some knot.
        """
        if system is not None:
            R_grid, E, M, mu = system.R_grid, system.E, system.M, system.mu
            jx = (system.jx_row, system.jx_col, system.jx_val)
        Rg = _host(R_grid, np.float64)
        Eh = _host(E, np.float64)
        is_dev = hasattr(M, "data_ptr")
        if is_dev:
            torch = self.torch
            cplx = M.is_complex()
            Mt = M.contiguous()
            Mt = Mt.to(torch.complex128 if cplx else torch.float64)
            M_ptr, mem = Mt.data_ptr(), MEM_DEVICE
            keep = Mt
        else:
            cplx = np.iscomplexobj(M)
            Mt = np.ascontiguousarray(M, dtype=np.complex128 if cplx else np.float64)
            M_ptr, mem = Mt.ctypes.data, MEM_HOST
            keep = Mt
        K, N = Rg.shape[0], Eh.shape[0]
        if tuple(Mt.shape) != (K, N, N):
            raise ValueError("M must be shaped [K, N, N] = [%d, %d, %d]" % (K, N, N))
        if storage is None:
            storage = "C128" if cplx else "R64"
        jr = jc = jv = None
        nnz = 0
        if jx is not None and len(jx[0]) > 0:
            jr, jc, jv = _host(jx[0], np.int32), _host(jx[1], np.int32), _host(jx[2], np.float64)
            nnz = jr.shape[0]
        d = SystemDesc(N, K, Rg.ctypes.data, Eh.ctypes.data, DTYPES["C128" if cplx else "R64"],
                       mem, M_ptr, DTYPES[storage], nnz, _ptr(jr), _ptr(jc), _ptr(jv), float(mu),
                       LAYOUTS[layout], float(drop_below))
        sid = C.c_int32()
        self._check(lib().mqct_system_load(self.h, C.byref(d), C.byref(sid)))
        del keep
        return sid.value

    def load_system_coo(self, *, R_grid, E, rows, cols, values, mu, jx=None, storage=None,
                        ld=None):
        """Upload a system given as a coordinate list of its coupling elements (both
        triangles): rows[i], cols[i] and values[k, i] at every knot k (hartree).
        rows, cols and values are numpy arrays (host) or CUDA tensors (device, all
        three); values real or complex, shaped [K, ld] with ld >= len(rows).
        Such a system runs decoupled (AT) dynamics on the "columns" schedule."""
        Rg = _host(R_grid, np.float64)
        Eh = _host(E, np.float64)
        K, N = Rg.shape[0], Eh.shape[0]
        is_dev = hasattr(values, "data_ptr")
        if is_dev:
            torch = self.torch
            cplx = values.is_complex()
            vt = values.contiguous().to(torch.complex128 if cplx else torch.float64)
            rt = rows.contiguous().to(torch.int32)
            ct = cols.contiguous().to(torch.int32)
            keep = (vt, rt, ct)
            mem = MEM_DEVICE
            vp_, rp_, cp_ = vt.data_ptr(), rt.data_ptr(), ct.data_ptr()
        else:
            cplx = np.iscomplexobj(values)
            vt = np.ascontiguousarray(values, dtype=np.complex128 if cplx else np.float64)
            rt, ct = _host(rows, np.int32), _host(cols, np.int32)
            keep = (vt, rt, ct)
            mem = MEM_HOST
            vp_, rp_, cp_ = vt.ctypes.data, rt.ctypes.data, ct.ctypes.data
        n_el = int(rt.shape[0])
        if ld is None:
            ld = int(vt.shape[-1])
        if vt.shape[0] != K or int(ct.shape[0]) != n_el:
            raise ValueError("values must be shaped [K, ld] and rows, cols [n_el]")
        if storage is None:
            storage = "C128" if cplx else "R64"
        jr = jc = jv = None
        nnz = 0
        if jx is not None and len(jx[0]) > 0:
            jr, jc, jv = _host(jx[0], np.int32), _host(jx[1], np.int32), _host(jx[2], np.float64)
            nnz = jr.shape[0]
        d = CooDesc(N, K, Rg.ctypes.data, Eh.ctypes.data, float(mu),
                    DTYPES["C128" if cplx else "R64"], mem, n_el, rp_, cp_, vp_, int(ld),
                    DTYPES[storage], nnz, _ptr(jr), _ptr(jc), _ptr(jv))
        sid = C.c_int32()
        self._check(lib().mqct_system_load_coo(self.h, C.byref(d), C.byref(sid)))
        del keep
        return sid.value

    def set_driver(self, sid, U):
        """Driving potential U(R_k) [K] (hartree) for AT dynamics on this system."""
        Uh = _host(U, np.float64)
        self._check(lib().mqct_system_set_driver(self.h, sid, Uh.ctypes.data))

    def system_bytes(self, sid):
        out = C.c_int64()
        self._check(lib().mqct_system_bytes(self.h, sid, C.byref(out)))
        return out.value

    def free_system(self, sid):
        self._check(lib().mqct_system_free(self.h, sid))

    # ------------------------------------------------------------------ batches
    def run(self, system_id, N_of, *, init_channel=None, a0=None, classical0=None, E_coll=None,
            b=None, R0=None, t0=None, dt=None, n_steps=None, integrator="rk4", rtol=1e-8,
            atol=1e-8, max_steps=100000, h_min=1e-6, schedule="auto", out=None,
            with_amplitudes=True, dynamics="ehrenfest", resume=False):
        """Propagate a batch; results are CUDA tensors filled asynchronously on the stream.

        system_id: [B] system ids; N_of: [B] channel count of each trajectory's system.
        resume=True continues every trajectory from the context's state store (the
        previous run's final states, or set_state's); RK4 then needs only n_steps.
        """
        torch = self.torch
        sid = _host(system_id, np.int32)
        B = int(sid.shape[0])
        Nof = np.asarray(N_of, np.int64).reshape(-1)
        total = int(Nof.sum())
        dev = self.device
        if out is None:
            out = {"P": torch.empty(total, dtype=torch.float64, device=dev),
                   "classical": torch.empty((B, 6), dtype=torch.float64, device=dev),
                   "t_final": torch.empty(B, dtype=torch.float64, device=dev),
                   "steps": torch.empty(B, dtype=torch.int64, device=dev),
                   "rejects": torch.empty(B, dtype=torch.int64, device=dev),
                   "status": torch.empty(B, dtype=torch.int32, device=dev),
                   "norm_err": torch.empty(B, dtype=torch.float64, device=dev),
                   "energy_err": torch.empty(B, dtype=torch.float64, device=dev),
                   "angmom_err": torch.empty(B, dtype=torch.float64, device=dev)}
            if with_amplitudes:
                out["a_final"] = torch.empty(total, dtype=torch.complex128, device=dev)
        a0h = None
        if a0 is not None:
            a0h = np.ascontiguousarray(np.asarray(a0, np.complex128).reshape(-1)).view(np.float64)
        c0h = None if classical0 is None else _host(np.reshape(classical0, (B, 6)), np.float64)
        bd = BatchDesc(
            B, sid.ctypes.data, None, _ptr(a0h), _ptr(c0h), None, None, None, None, INTEGRATORS[integrator], None, None,
            float(rtol), float(atol), int(max_steps), float(h_min), SCHEDULES[schedule],
            DYNAMICS[dynamics], 1 if resume else 0)
        hold = []
        for name, arr, dtp in (("init_channel", init_channel, np.int32), ("E_coll", E_coll, np.float64),
                               ("b", b, np.float64), ("R0", R0, np.float64), ("t0", t0, np.float64),
                               ("dt", dt, np.float64), ("n_steps", n_steps, np.int64)):
            if arr is None:
                continue
            h = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtp), (B,)))
            hold.append(h)
            setattr(bd, name, h.ctypes.data)
        res = BatchResult(MEM_DEVICE, _ptr(out.get("P")), _ptr(out.get("a_final")),
                          _ptr(out.get("classical")), _ptr(out.get("t_final")),
                          _ptr(out.get("steps")), _ptr(out.get("rejects")),
                          _ptr(out.get("status")), _ptr(out.get("norm_err")),
                          _ptr(out.get("energy_err")), _ptr(out.get("angmom_err")))
        self._check(lib().mqct_run(self.h, C.byref(bd), C.byref(res)))
        return out

    def run_noalloc(self, system_id, out, *, init_channel=None, a0=None, classical0=None,
                    E_coll=None, b=None, R0=None, t0=None, dt=None, n_steps=None,
                    dynamics="ehrenfest"):
        """mqct_run_noalloc: fixed-step RK4 on the per-trajectory schedule into the
        caller's CUDA tensors `out` (keys as run() returns; P required), with no
        device allocation by the library."""
        sid = _host(system_id, np.int32)
        B = int(sid.shape[0])
        a0h = None
        if a0 is not None:
            a0h = np.ascontiguousarray(np.asarray(a0, np.complex128).reshape(-1)).view(np.float64)
        c0h = None if classical0 is None else _host(np.reshape(classical0, (B, 6)), np.float64)
        bd = BatchDesc(B, sid.ctypes.data, None, _ptr(a0h), _ptr(c0h), None, None, None, None,
                       INTEGRATORS["rk4"], None, None, 0.0, 0.0, 0, 0.0, SCHEDULES["gemv"],
                       DYNAMICS[dynamics], 0)
        hold = []
        for name, arr, dtp in (("init_channel", init_channel, np.int32), ("E_coll", E_coll, np.float64),
                               ("b", b, np.float64), ("R0", R0, np.float64), ("t0", t0, np.float64),
                               ("dt", dt, np.float64), ("n_steps", n_steps, np.int64)):
            if arr is None:
                continue
            h = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtp), (B,)))
            hold.append(h)
            setattr(bd, name, h.ctypes.data)
        res = BatchResult(MEM_DEVICE, _ptr(out.get("P")), _ptr(out.get("a_final")),
                          _ptr(out.get("classical")), _ptr(out.get("t_final")),
                          _ptr(out.get("steps")), _ptr(out.get("rejects")),
                          _ptr(out.get("status")), _ptr(out.get("norm_err")),
                          _ptr(out.get("energy_err")), _ptr(out.get("angmom_err")))
        self._check(lib().mqct_run_noalloc(self.h, C.byref(bd), C.byref(res)))
        return out

    def run_host(self, system_id, N_of, **kw):
        """As run(), with host (numpy) results; returns after they are filled."""
        sid = _host(system_id, np.int32)
        B = int(sid.shape[0])
        total = int(np.asarray(N_of, np.int64).sum())
        out = {"P": np.empty(total), "a_final": np.empty(total, np.complex128),
               "classical": np.empty((B, 6)), "t_final": np.empty(B),
               "steps": np.empty(B, np.int64), "rejects": np.empty(B, np.int64),
               "status": np.empty(B, np.int32), "norm_err": np.empty(B),
               "energy_err": np.empty(B), "angmom_err": np.empty(B)}
        kw = dict(kw)
        schedule = kw.pop("schedule", "auto")
        integrator = kw.pop("integrator", "rk4")
        dynamics = kw.pop("dynamics", "ehrenfest")
        resume = kw.pop("resume", False)
        a0 = kw.pop("a0", None)
        classical0 = kw.pop("classical0", None)
        a0h = None
        if a0 is not None:
            a0h = np.ascontiguousarray(np.asarray(a0, np.complex128).reshape(-1)).view(np.float64)
        c0h = None if classical0 is None else _host(np.reshape(classical0, (B, 6)), np.float64)
        bd = BatchDesc(B, sid.ctypes.data, None, _ptr(a0h), _ptr(c0h), None, None, None, None,
                       INTEGRATORS[integrator], None, None, float(kw.pop("rtol", 1e-8)),
                       float(kw.pop("atol", 1e-8)), int(kw.pop("max_steps", 100000)),
                       float(kw.pop("h_min", 1e-6)), SCHEDULES[schedule], DYNAMICS[dynamics],
                       1 if resume else 0)
        hold = []
        for name, dtp in (("init_channel", np.int32), ("E_coll", np.float64), ("b", np.float64),
                          ("R0", np.float64), ("t0", np.float64), ("dt", np.float64),
                          ("n_steps", np.int64)):
            arr = kw.pop(name, None)
            if arr is None:
                continue
            h = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtp), (B,)))
            hold.append(h)
            setattr(bd, name, h.ctypes.data)
        if kw:
            raise TypeError("unknown arguments: %s" % sorted(kw))
        res = BatchResult(MEM_HOST, *[out[k].ctypes.data for k in
                                      ("P", "a_final", "classical", "t_final", "steps", "rejects",
                                       "status", "norm_err", "energy_err", "angmom_err")])
        self._check(lib().mqct_run(self.h, C.byref(bd), C.byref(res)))
        return out

    # ------------------------------------------------------------------ state store
    def get_state(self, first=0, count=None):
        """Host copies of the stored states of trajectories [first, first + count)
        (default: all of the last run): (records as a STATE_DTYPE array, amplitudes
        as one complex array concatenated in batch order)."""
        if count is None:
            count = self.stored_count() - first
        rec = np.zeros(count, STATE_DTYPE)
        self._check(lib().mqct_get_state(self.h, int(first), int(count), rec.ctypes.data, None))
        amps = np.empty(int(rec["N"].sum()), np.complex128)
        self._check(lib().mqct_get_state(self.h, int(first), int(count), rec.ctypes.data,
                                         amps.ctypes.data))
        return rec, amps

    def set_state(self, rec, amps, first=0):
        """Write states (STATE_DTYPE records and their concatenated amplitudes) into
        the store; with first = 0 and a different count the store is redefined."""
        rec = np.ascontiguousarray(rec, STATE_DTYPE)
        a = np.ascontiguousarray(np.asarray(amps, np.complex128).reshape(-1))
        if a.shape[0] != int(rec["N"].sum()):
            raise ValueError("set_state: %d amplitudes for records holding %d channels"
                             % (a.shape[0], int(rec["N"].sum())))
        self._check(lib().mqct_set_state(self.h, int(first), rec.shape[0], rec.ctypes.data,
                                         a.ctypes.data))

    def stored_count(self):
        """Number of trajectories in the state store."""
        n = C.c_int64()
        self._check(lib().mqct_state_count(self.h, C.byref(n)))
        return n.value

    # ------------------------------------------------------------------ gradients
    def set_params(self, sid, radial, gidx, G):
        """Attach the linear parametric form M(R_k) = sum_p theta_p radial[p][k] G[gidx[p]]."""
        rad = _host(radial, np.float64)
        gi = _host(gidx, np.int32)
        Gh = _host(G, np.float64)
        self._check(lib().mqct_system_set_params(self.h, sid, rad.shape[0], rad.ctypes.data,
                                                 gi.ctypes.data, Gh.shape[0], Gh.ctypes.data))
        self._nparam = rad.shape[0]

    def set_theta(self, sid, theta):
        """Rebuild the system's tables on the device at the coefficients theta."""
        th = _host(theta, np.float64)
        self._check(lib().mqct_system_set_theta(self.h, sid, th.ctypes.data))

    def adjoint(self, sid, N, dL_dP, *, init_channel, E_coll, b, dt, n_steps, R0=None,
                checkpoint_every=256, n_param=None):
        """dL/dtheta of L = sum dL_dP * P (host arrays); returns (grad, P)."""
        B = len(np.atleast_1d(E_coll))
        sids = np.full(B, sid, np.int32)
        hold = []
        bd = BatchDesc(B, sids.ctypes.data, None, None, None, None, None, None, None, 0, None,
                       None, 0.0, 0.0, 0, 0.0, 0, 0)
        for name, arr, dtp in (("init_channel", init_channel, np.int32), ("E_coll", E_coll, np.float64),
                               ("b", b, np.float64), ("R0", R0, np.float64), ("dt", dt, np.float64),
                               ("n_steps", n_steps, np.int64)):
            if arr is None:
                continue
            h = np.ascontiguousarray(np.broadcast_to(np.asarray(arr, dtp), (B,)))
            hold.append(h)
            setattr(bd, name, h.ctypes.data)
        w = _host(np.reshape(dL_dP, -1), np.float64)
        P = np.empty(B * N)
        g = np.empty(n_param if n_param is not None else self._nparam)
        self._check(lib().mqct_adjoint(self.h, C.byref(bd), int(checkpoint_every), w.ctypes.data,
                                       g.ctypes.data, P.ctypes.data))
        return g, P.reshape(B, N)

    def build_couplings(self, basis, expansion, tables=True, angular=False):
        """Coupling matrices of an asymmetric top + linear rotor (Eqs. 12-18) on the GPU.

        basis: channels j, m, rot1, j2 and rotor-1 states rot1_j, b (b_k at column
        k + j1); expansion: terms lam1, mu1, lam2, lam and radial coefficients v[T, K]
        (hartree).  Returns {"M": [K, N, N]} and/or {"G": [T, N, N]} as FP64 CUDA
        tensors, ready for load_system(M=...) and set_params."""
        torch = self.torch
        i32 = lambda a: _host(a, np.int32)
        j, m, r1, j2 = i32(basis.j), i32(basis.m), i32(basis.rot1), i32(basis.j2)
        rj, b = i32(basis.rot1_j), _host(basis.b, np.float64)
        l1, u1, l2, l = (i32(expansion.lam1), i32(expansion.mu1), i32(expansion.lam2),
                         i32(expansion.lam))
        v = _host(expansion.v, np.float64)
        N, T, K = j.shape[0], l1.shape[0], v.shape[1]
        out = {}
        if tables:
            out["M"] = torch.empty((K, N, N), dtype=torch.float64, device=self.device)
        if angular:
            out["G"] = torch.empty((T, N, N), dtype=torch.float64, device=self.device)
        d = CouplingDesc(N, _ptr(j), _ptr(m), _ptr(r1), _ptr(j2), rj.shape[0], _ptr(rj),
                         _ptr(b), b.shape[1], T, _ptr(l1), _ptr(u1), _ptr(l2), _ptr(l), K,
                         _ptr(v))
        self._check(lib().mqct_coupling_build(self.h, C.byref(d), _ptr(out.get("M")),
                                              _ptr(out.get("G"))))
        return out

    def build_couplings_sparse(self, basis, expansion, v_screen, drop_below, capacity=None):
        """Screened build (mqct_coupling_build_sparse): the equal-m elements whose
        largest |M| at the screening radii (v_screen [T, S], hartree) exceeds
        drop_below, as device tensors rows [n], cols [n] (int32) and values [K, n]
        (FP64).  capacity None: count first, then build with the exact capacity."""
        torch = self.torch
        i32 = lambda a: _host(a, np.int32)
        j, m, r1, j2 = i32(basis.j), i32(basis.m), i32(basis.rot1), i32(basis.j2)
        rj, b = i32(basis.rot1_j), _host(basis.b, np.float64)
        l1, u1, l2, l = (i32(expansion.lam1), i32(expansion.mu1), i32(expansion.lam2),
                         i32(expansion.lam))
        v = _host(expansion.v, np.float64)
        vs = _host(v_screen, np.float64)
        N, T, K = j.shape[0], l1.shape[0], v.shape[1]
        d = CouplingDesc(N, _ptr(j), _ptr(m), _ptr(r1), _ptr(j2), rj.shape[0], _ptr(rj),
                         _ptr(b), b.shape[1], T, _ptr(l1), _ptr(u1), _ptr(l2), _ptr(l), K,
                         _ptr(v))
        n = C.c_int64()
        if capacity is None:
            code = lib().mqct_coupling_build_sparse(self.h, C.byref(d), vs.shape[1], _ptr(vs),
                                                    float(drop_below), 0, None, None, None,
                                                    C.byref(n))
            if code not in (OK, ERR_ARG) or (code == ERR_ARG and n.value == 0):
                self._check(code)
            capacity = n.value
        cap = max(int(capacity), 1)
        rows = torch.empty(cap, dtype=torch.int32, device=self.device)
        cols = torch.empty(cap, dtype=torch.int32, device=self.device)
        vals = torch.empty((K, cap), dtype=torch.float64, device=self.device)
        self._check(lib().mqct_coupling_build_sparse(self.h, C.byref(d), vs.shape[1], _ptr(vs),
                                                     float(drop_below), cap, _ptr(rows),
                                                     _ptr(cols), _ptr(vals), C.byref(n)))
        k = n.value
        return {"rows": rows[:k], "cols": cols[:k], "values": vals[:, :k], "n_kept": k}

    def xs_symmetrize(self, sigma, g):
        """Eq. 19 ratio and Eq. 20 symmetrised cross sections of sigma[n_E, L, L]
        (host arrays in, host arrays out; computed on the GPU)."""
        sigma = _host(sigma, np.float64)
        g = _host(g, np.float64)
        nE, L = sigma.shape[0], sigma.shape[1]
        sym = np.empty_like(sigma)
        ratio = np.empty_like(sigma)
        self._check(lib().mqct_xs_symmetrize(self.h, MEM_HOST, nE, L, _ptr(g), _ptr(sigma),
                                             _ptr(sym), _ptr(ratio)))
        return sym, ratio

    def rate_coefficients(self, U, sym, E_level, g, mu, beta):
        """k[n_T, L, L] (bohr^3 per a.u. of time) from the symmetrised cross sections
        sym[n_E, L, L] at the energies U[n_E]; beta = k_B T (hartree)."""
        U, sym, E, g, beta = (_host(a, np.float64) for a in (U, sym, E_level, g, beta))
        nE, L, nT = sym.shape[0], sym.shape[1], beta.shape[0]
        k = np.empty((nT, L, L))
        self._check(lib().mqct_rate_coefficients(self.h, MEM_HOST, nE, L, _ptr(U), _ptr(E),
                                                 _ptr(g), _ptr(sym), float(mu), nT, _ptr(beta),
                                                 _ptr(k)))
        return k

    def set_option(self, name, value=1):
        """Schedule options: graphs, autotune, chunk, reset_tuning, tail, per_launch (the work list);
        col_workspace (the columns schedule's workspace cap in bytes, 0 = default)."""
        self._check(lib().mqct_set_option(self.h, OPTIONS[name], int(value)))

    def tuning_report(self):
        """The autotuner's shape choices so far (parsed JSON)."""
        import json
        return json.loads(lib().mqct_tuning_report(self.h).decode())

    def set_profiling(self, enable=True):
        """Time the dominant step kernel of later runs with HIP events."""
        self._check(lib().mqct_set_profiling(self.h, 1 if enable else 0))

    def profile_read(self, with_bytes=False):
        """(total milliseconds, launches) of the timed kernel since the last read, and
        with_bytes=True also the algorithmic table bytes those launches read."""
        ms, n, by = C.c_double(), C.c_int64(), C.c_double()
        self._check(lib().mqct_profile_read(self.h, C.byref(ms), C.byref(n), C.byref(by)))
        if with_bytes:
            return ms.value, n.value, by.value
        return ms.value, n.value

    def read_bandwidth(self, buf, reps=20):
        """Mean milliseconds of one streaming read of the device tensor `buf` (the
        measured read reference for bandwidth-bound kernels)."""
        ms = C.c_double()
        self._check(lib().mqct_read_bandwidth(self.h, C.c_void_p(buf.data_ptr()),
                                              buf.numel() * buf.element_size(), int(reps),
                                              C.byref(ms)))
        return ms.value

    def cross_sections(self, P, b, init_level, level_of_channel, n_levels, b_max):
        """Monte-Carlo cross sections (bohr^2) from P [B, N] on the device."""
        torch = self.torch
        P = P.contiguous()
        B, N = P.shape
        bt = torch.as_tensor(np.asarray(b, np.float64), device=self.device)
        il = torch.as_tensor(np.asarray(init_level, np.int32), device=self.device)
        lev = _host(level_of_channel, np.int32)
        sig = torch.empty((n_levels, n_levels), dtype=torch.float64, device=self.device)
        self._check(lib().mqct_cross_sections(self.h, MEM_DEVICE, B, N, P.data_ptr(),
                                              bt.data_ptr(), il.data_ptr(), lev.ctypes.data,
                                              int(n_levels), float(b_max), sig.data_ptr()))
        return sig


# batch keys whose forward computation the adjoint differentiates: fixed-step RK4
# from init_channel / E_coll / b / R0 (mean-field dynamics, any schedule)
ADJOINT_KEYS = ("init_channel", "E_coll", "b", "R0", "dt", "n_steps", "schedule")


def _check_adjoint_batch(batch):
    """Raise unless the backward pass differentiates exactly the forward's batch."""
    extra = sorted(k for k in batch if k not in ADJOINT_KEYS and batch[k] is not None)
    for k, ok in (("integrator", "rk4"), ("dynamics", "ehrenfest")):
        if k in extra and batch[k] == ok:
            extra.remove(k)
    if extra:
        raise ValueError("the adjoint differentiates fixed-step RK4 mean-field batches started "
                         "from init_channel / E_coll / b / R0; unsupported batch keys: %s"
                         % ", ".join(extra))
    for k in ("init_channel", "E_coll", "b", "dt", "n_steps"):
        if batch.get(k) is None:
            raise ValueError("the adjoint needs batch[%r]" % k)


def _autograd_function():
    import torch

    class MQCTPropagate(torch.autograd.Function):
        """P = propagate(theta): final probabilities [B, N] of an RK4 batch as a function of
        the potential coefficients theta; backward runs the library's adjoint kernel."""

        @staticmethod
        def forward(fctx, theta, mq, sid, N, batch, checkpoint_every):
            _check_adjoint_batch(batch)
            th = theta.detach().cpu().double().numpy()
            mq.set_theta(sid, th)
            B = len(batch["E_coll"])
            out = mq.run_host([sid] * B, [N] * B, **batch)
            fctx.mq, fctx.sid, fctx.N, fctx.batch, fctx.S = mq, sid, N, batch, checkpoint_every
            fctx.save_for_backward(theta)
            return torch.as_tensor(out["P"].reshape(B, N), dtype=theta.dtype, device=theta.device)

        @staticmethod
        def backward(fctx, grad_P):
            (theta,) = fctx.saved_tensors
            mq = fctx.mq
            mq.set_theta(fctx.sid, theta.detach().cpu().double().numpy())
            b = fctx.batch
            g, _ = mq.adjoint(fctx.sid, fctx.N, grad_P.detach().cpu().double().numpy(),
                              init_channel=b["init_channel"], E_coll=b["E_coll"], b=b["b"],
                              dt=b["dt"], n_steps=b["n_steps"], R0=b.get("R0"),
                              checkpoint_every=fctx.S, n_param=theta.numel())
            return (torch.as_tensor(g, dtype=theta.dtype, device=theta.device),
                    None, None, None, None, None)

    return MQCTPropagate


def propagate(theta, mq, sid, N, batch, checkpoint_every=256):
    """Differentiable final probabilities (see MQCTPropagate)."""
    return _autograd_function().apply(theta, mq, sid, N, batch, checkpoint_every)
