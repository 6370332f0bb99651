"""Python binding of the OSCAR HIP library (liboscar.so, C ABI of
include/oscar.h).  Argument marshalling only: every step of the relaxation
path runs in the library's HIP kernels.  PyTorch supplies the device
workspace and the stream."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboscar.so")

OK, W_PCG_MAXIT, W_REFINE_STALL = 0, 1, 2
E_ARG, E_WORKSPACE, E_MASK, E_UNSTABLE, E_NONFINITE, E_HIP, E_CAPACITY = -1, -2, -3, -4, -5, -6, -7
FP64, MIXED = 0, 1
PC_JACOBI, PC_MG = 0, 1
SOLVE_DEFAULT, SOLVE_LAUNCHES, SOLVE_PERSISTENT = 0, 1, 2
FIELDS = dict(alpha=0, U=1, p=2, U_vd=3, p_vd=4, U_cr=5, p_cr=6, phi_vd=7, phi_vd_prev=8, phi_cr=9,
              kappa=10, rAU=11, rhs=12, U_sum=13, HbyA=14, nhatf=15)

EXPORTS = ["oscar_workspace_size", "oscar_create", "oscar_create_static", "oscar_viscous_step", "oscar_capillary_relax",
           "oscar_relax_history", "oscar_pressure_solve", "oscar_get_field", "oscar_set_field",
           "oscar_field_len", "oscar_stats", "oscar_destroy", "oscar_last_error", "oscar_dt_brackbill",
           "oscar_timing", "oscar_timing_read"]


class Desc(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("mask", C.POINTER(C.c_uint8)), ("alpha0", C.POINTER(C.c_double)),
                ("rho1", C.c_double), ("mu1", C.c_double), ("rho2", C.c_double), ("mu2", C.c_double),
                ("sigma", C.c_double), ("theta_deg", C.c_double), ("bc", C.c_int32 * 6),
                ("u_inlet", C.c_double), ("precision", C.c_int32), ("n_corr", C.c_int32),
                ("pcg_rtol", C.c_double), ("pcg_max_it", C.c_int32), ("precond", C.c_int32),
                ("mules_iter", C.c_int32), ("mg_sweeps2", C.c_int32), ("max_blocks", C.c_int32),
                ("inner_rtol", C.c_double), ("solve_mode", C.c_int32), ("reserved", C.c_int32)]


class Stats(C.Structure):
    _fields_ = [("mass_phase1", C.c_double), ("max_courant", C.c_double), ("mass_defect", C.c_double),
                ("last_E", C.c_double), ("last_res", C.c_double), ("last_pcg_iters", C.c_int32),
                ("pcg_iters_call", C.c_int32), ("refine_steps_call", C.c_int32), ("k_f", C.c_int32),
                ("n_fluid", C.c_int32), ("pcg_maxit_hits", C.c_int32)]


class OscarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("OSCAR error %d: %s" % (code, msg))
        self.code = code


_lib = None


def lib():
    """Load liboscar.so; raises if the HIP library has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise OSError("liboscar.so is not built (run __graft_entry__.build() or "
                          "python paper_2105_10576_amd/build.py)")
        L = C.CDLL(LIB_PATH)
        dp, ip, vp = C.POINTER(C.c_double), C.POINTER(C.c_int32), C.c_void_p
        L.oscar_workspace_size.argtypes = [C.POINTER(Desc), C.POINTER(C.c_uint64)]
        L.oscar_create.argtypes = [C.POINTER(Desc), vp, C.c_uint64, vp, C.POINTER(vp)]
        L.oscar_create_static.argtypes = [C.POINTER(Desc), vp, C.POINTER(vp)]
        L.oscar_viscous_step.argtypes = [vp, C.c_double]
        L.oscar_capillary_relax.argtypes = [vp, C.c_double, C.c_int32, C.c_int32, C.c_double, ip, dp]
        L.oscar_relax_history.argtypes = [vp, dp, C.c_int32, ip]
        L.oscar_pressure_solve.argtypes = [vp, C.c_int32, C.c_double, C.c_double, C.c_int32, ip, dp]
        L.oscar_get_field.argtypes = [vp, C.c_int32, dp]
        L.oscar_set_field.argtypes = [vp, C.c_int32, dp]
        L.oscar_field_len.argtypes = [vp, C.c_int32]
        L.oscar_field_len.restype = C.c_int64
        L.oscar_stats.argtypes = [vp, C.POINTER(Stats)]
        L.oscar_destroy.argtypes = [vp]
        L.oscar_destroy.restype = None
        L.oscar_last_error.argtypes = [vp]
        L.oscar_last_error.restype = C.c_char_p
        L.oscar_dt_brackbill.argtypes = [C.c_double] * 4
        L.oscar_dt_brackbill.restype = C.c_double
        L.oscar_timing.argtypes = [vp, C.c_int32]
        L.oscar_timing.restype = C.c_int32
        L.oscar_timing_read.argtypes = [vp, C.c_int32, dp, C.POINTER(C.c_int64)]
        L.oscar_timing_read.restype = C.c_int32
        for name in ("oscar_workspace_size", "oscar_create", "oscar_create_static", "oscar_viscous_step",
                     "oscar_capillary_relax", "oscar_relax_history", "oscar_pressure_solve", "oscar_get_field", "oscar_set_field",
                     "oscar_stats"):
            getattr(L, name).restype = C.c_int32
        _lib = L
    return _lib


def make_desc(case, precision=FP64):
    """Fill an oscar_desc from a case dictionary (key "precond": PC_JACOBI,
    the default, or PC_MG; key "mules_iter": limiting passes of the alpha
    transport, default 1; tuning keys "mg_sweeps2", "max_blocks",
    "inner_rtol", default 0 = the library's built-in value; key
    "solve_mode": SOLVE_*, default SOLVE_DEFAULT); returns (desc,
    keep-alive arrays)."""
    d = Desc()
    for k in ("dim", "nx", "ny", "nz", "n_corr", "pcg_max_it"):
        setattr(d, k, int(case[k]))
    for k in ("h", "rho1", "mu1", "rho2", "mu2", "sigma", "theta_deg", "u_inlet", "pcg_rtol"):
        setattr(d, k, float(case[k]))
    for i in range(6):
        d.bc[i] = int(case["bc"][i])
    d.precision = int(precision)
    d.precond = int(case.get("precond", PC_JACOBI))
    d.mules_iter = int(case.get("mules_iter", 1))
    d.mg_sweeps2 = int(case.get("mg_sweeps2", 0))
    d.max_blocks = int(case.get("max_blocks", 0))
    d.inner_rtol = float(case.get("inner_rtol", 0.0))
    d.solve_mode = int(case.get("solve_mode", SOLVE_DEFAULT))
    mask = np.ascontiguousarray(case["mask"], dtype=np.uint8)
    a0 = np.ascontiguousarray(case["alpha0"], dtype=np.float64)
    d.mask = mask.ctypes.data_as(C.POINTER(C.c_uint8))
    d.alpha0 = a0.ctypes.data_as(C.POINTER(C.c_double))
    return d, (mask, a0)


def workspace_size(case, precision=FP64):
    d, keep = make_desc(case, precision)
    n = C.c_uint64(0)
    rc = lib().oscar_workspace_size(C.byref(d), C.byref(n))
    if rc != OK:
        raise OscarError(rc, lib().oscar_last_error(None).decode())
    return n.value


def dt_brackbill(rho1, rho2, h, sigma):
    return lib().oscar_dt_brackbill(rho1, rho2, h, sigma)


class Oscar:
    """One OSCAR context on a GPU; fields stay resident in a torch uint8
    workspace tensor on that device, or (static_workspace=True) in the
    library's static device array (oscar_create_static: no allocation)."""

    def __init__(self, case, precision=FP64, device="cuda:0", stream=None, static_workspace=False, **over):
        import torch

        c = dict(case)
        c.update(over)
        self.case = c
        self.precision = precision
        self.device = torch.device(device)
        d, keep = make_desc(c, precision)
        n = C.c_uint64(0)
        L = lib()
        rc = L.oscar_workspace_size(C.byref(d), C.byref(n))
        if rc != OK:
            raise OscarError(rc, L.oscar_last_error(None).decode())
        self.ws_bytes = n.value
        self.ws = None if static_workspace else torch.empty(self.ws_bytes, dtype=torch.uint8, device=self.device)
        if stream is None:
            stream = torch.cuda.current_stream(self.device)
        self.stream = stream
        self.ctx = C.c_void_p(None)
        with torch.cuda.device(self.device):
            if static_workspace:
                rc = L.oscar_create_static(C.byref(d), C.c_void_p(stream.cuda_stream), C.byref(self.ctx))
            else:
                rc = L.oscar_create(C.byref(d), C.c_void_p(self.ws.data_ptr()), self.ws_bytes,
                                    C.c_void_p(stream.cuda_stream), C.byref(self.ctx))
        if rc != OK:
            raise OscarError(rc, L.oscar_last_error(None).decode())
        self.nc = int(c["nx"]) * int(c["ny"]) * int(c["nz"])
        self.dim = int(c["dim"])

    def close(self):
        if getattr(self, "ctx", None) and self.ctx.value:
            lib().oscar_destroy(self.ctx)
            self.ctx = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, allow=(OK, W_PCG_MAXIT, W_REFINE_STALL)):
        if rc not in allow:
            raise OscarError(rc, lib().oscar_last_error(self.ctx).decode())
        return rc

    def viscous_step(self, dt_vd, check=True):
        rc = lib().oscar_viscous_step(self.ctx, float(dt_vd))
        return self._check(rc) if check else rc

    def capillary_relax(self, dt_vd, n_sub, max_iters, tol, check=True):
        kf = C.c_int32(0)
        E = C.c_double(0.0)
        rc = lib().oscar_capillary_relax(self.ctx, float(dt_vd), int(n_sub), int(max_iters), float(tol),
                                         C.byref(kf), C.byref(E))
        if check:
            self._check(rc)
        return rc, kf.value, self.relax_history()

    def relax_history(self):
        buf = np.zeros(4096)
        n = C.c_int32(0)
        lib().oscar_relax_history(self.ctx, buf.ctypes.data_as(C.POINTER(C.c_double)), 4096, C.byref(n))
        return buf[:n.value].copy()

    def step(self, dt_vd=None, n_sub=None, max_iters=None, tol=None):
        c = self.case
        dt_vd = c["dt_vd"] if dt_vd is None else dt_vd
        n_sub = c["n_sub"] if n_sub is None else n_sub
        max_iters = c["max_iters"] if max_iters is None else max_iters
        tol = c["tol"] if tol is None else tol
        rc1 = self.viscous_step(dt_vd)
        rc2, kf, E = self.capillary_relax(dt_vd, n_sub, max_iters, tol)
        return rc1, rc2, kf, E

    def pressure_solve(self, which, dt, rtol, max_it):
        it = C.c_int32(0)
        res = C.c_double(0.0)
        rc = lib().oscar_pressure_solve(self.ctx, int(which), float(dt), float(rtol), int(max_it),
                                        C.byref(it), C.byref(res))
        self._check(rc)
        return rc, it.value, res.value

    def get(self, name):
        fid = FIELDS[name]
        n = lib().oscar_field_len(self.ctx, fid)
        out = np.empty(n, dtype=np.float64)
        self._check(lib().oscar_get_field(self.ctx, fid, out.ctypes.data_as(C.POINTER(C.c_double))))
        return out

    def set(self, name, arr):
        fid = FIELDS[name]
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.size == lib().oscar_field_len(self.ctx, fid)
        self._check(lib().oscar_set_field(self.ctx, fid, a.ctypes.data_as(C.POINTER(C.c_double))))

    def timing(self, period):
        """period >= 1: bracket every period-th CG iteration (True = 1); 0 / False: stop."""
        self._check(lib().oscar_timing(self.ctx, int(period)))

    def timing_read(self, kernel):
        ms = C.c_double(0.0)
        n = C.c_int64(0)
        self._check(lib().oscar_timing_read(self.ctx, int(kernel), C.byref(ms), C.byref(n)))
        return ms.value, n.value

    def stats(self):
        s = Stats()
        self._check(lib().oscar_stats(self.ctx, C.byref(s)))
        return {k: getattr(s, k) for k, _ in Stats._fields_}


ENGINE_EXPORTS = ["oscar_engine_table_bytes", "oscar_engine_create", "oscar_engine_admit", "oscar_engine_run",
                  "oscar_engine_poll", "oscar_engine_fetch", "oscar_engine_release", "oscar_engine_free_bytes",
                  "oscar_engine_stats", "oscar_engine_destroy", "oscar_engine_last_error",
                  "oscar_engine_set_solve_mode"]
EXPORTS = EXPORTS + ENGINE_EXPORTS


def _engine_sigs(L):
    vp, ip = C.c_void_p, C.POINTER(C.c_int32)
    dp = C.POINTER(C.c_double)
    L.oscar_engine_table_bytes.argtypes = [C.c_int32, C.POINTER(C.c_uint64)]
    L.oscar_engine_create.argtypes = [C.c_int32, C.c_int32, vp, C.c_uint64, vp, C.POINTER(vp)]
    L.oscar_engine_admit.argtypes = [vp, C.POINTER(Desc), C.c_double, C.c_int32, C.c_int32, C.c_double, ip]
    L.oscar_engine_run.argtypes = [vp, C.c_int32]
    L.oscar_engine_set_solve_mode.argtypes = [vp, C.c_int32]
    L.oscar_engine_poll.argtypes = [vp, ip, C.c_int32, ip, ip]
    L.oscar_engine_fetch.argtypes = [vp, C.c_int32, dp, dp, dp, ip, ip]
    L.oscar_engine_release.argtypes = [vp, C.c_int32]
    L.oscar_engine_free_bytes.argtypes = [vp, C.POINTER(C.c_uint64), ip]
    L.oscar_engine_stats.argtypes = [vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)]
    L.oscar_engine_destroy.argtypes = [vp]
    L.oscar_engine_destroy.restype = None
    L.oscar_engine_last_error.argtypes = [vp]
    L.oscar_engine_last_error.restype = C.c_char_p
    for n in ENGINE_EXPORTS:
        if n not in ("oscar_engine_destroy", "oscar_engine_last_error"):
            getattr(L, n).restype = C.c_int32


def engine_table_bytes(max_slots):
    L = lib()
    _engine_sigs(L)
    n = C.c_uint64(0)
    rc = L.oscar_engine_table_bytes(int(max_slots), C.byref(n))
    if rc != OK:
        raise OscarError(rc, L.oscar_last_error(None).decode())
    return n.value


class Engine:
    """Continuous-batching engine over one torch device workspace of
    table bytes + heap_bytes (the HBM budget for resident requests)."""

    def __init__(self, max_slots, heap_bytes, precision=FP64, device="cuda:0", stream=None, solve_mode=SOLVE_DEFAULT):
        import torch

        L = lib()
        _engine_sigs(L)
        self.precision = precision
        self.max_slots = int(max_slots)
        self.table = engine_table_bytes(max_slots)
        self.bytes = self.table + int(heap_bytes)
        self.ws = torch.empty(self.bytes, dtype=torch.uint8, device=device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(torch.device(device))
        self.h = C.c_void_p(None)
        with torch.cuda.device(torch.device(device)):
            rc = L.oscar_engine_create(self.max_slots, int(precision), C.c_void_p(self.ws.data_ptr()), self.bytes,
                                       C.c_void_p(self.stream.cuda_stream), C.byref(self.h))
        if rc != OK:
            raise OscarError(rc, L.oscar_last_error(None).decode())
        self.meta = {}
        if solve_mode != SOLVE_DEFAULT:
            self.set_solve_mode(solve_mode)

    def set_solve_mode(self, mode):
        """SOLVE_LAUNCHES or SOLVE_PERSISTENT from the next tick on."""
        rc = lib().oscar_engine_set_solve_mode(self.h, int(mode))
        if rc != OK:
            self._err(rc)

    def close(self):
        if getattr(self, "h", None) and self.h.value:
            lib().oscar_engine_destroy(self.h)
            self.h = C.c_void_p(None)

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _err(self, rc):
        raise OscarError(rc, lib().oscar_engine_last_error(self.h).decode())

    def admit(self, case, dt_vd=None, n_sub=None, max_iters=None, tol=None):
        """Admit a request; returns the slot, or None when it does not fit now."""
        d, keep = make_desc(case, self.precision)
        slot = C.c_int32(-1)
        rc = lib().oscar_engine_admit(self.h, C.byref(d), float(case["dt_vd"] if dt_vd is None else dt_vd),
                                      int(case["n_sub"] if n_sub is None else n_sub),
                                      int(case["max_iters"] if max_iters is None else max_iters),
                                      float(case["tol"] if tol is None else tol), C.byref(slot))
        if rc == E_CAPACITY:
            return None
        if rc != OK:
            self._err(rc)
        self.meta[slot.value] = (int(case["nx"]) * int(case["ny"]) * int(case["nz"]), int(case["dim"]))
        return slot.value

    def run(self, ticks=1):
        rc = lib().oscar_engine_run(self.h, int(ticks))
        if rc != OK:
            self._err(rc)

    def poll(self):
        buf = (C.c_int32 * self.max_slots)()
        n = C.c_int32(0)
        a = C.c_int32(0)
        lib().oscar_engine_poll(self.h, buf, self.max_slots, C.byref(n), C.byref(a))
        return [buf[i] for i in range(n.value)], a.value

    def fetch(self, slot):
        nc, dim = self.meta[slot]
        alpha = np.empty(nc)
        p = np.empty(nc)
        U = np.empty(dim * nc)
        kf = C.c_int32(0)
        st = C.c_int32(0)
        dp = C.POINTER(C.c_double)
        rc = lib().oscar_engine_fetch(self.h, int(slot), alpha.ctypes.data_as(dp), p.ctypes.data_as(dp),
                                      U.ctypes.data_as(dp), C.byref(kf), C.byref(st))
        if rc != OK:
            self._err(rc)
        return dict(alpha=alpha, p=p, U=U, k_f=kf.value, status=st.value)

    def release(self, slot):
        rc = lib().oscar_engine_release(self.h, int(slot))
        if rc != OK:
            self._err(rc)
        self.meta.pop(slot, None)

    def free(self):
        m = C.c_uint64(0)
        f = C.c_int32(0)
        lib().oscar_engine_free_bytes(self.h, C.byref(m), C.byref(f))
        return m.value, f.value

    def stats(self):
        t = C.c_int64(0)
        it = C.c_int64(0)
        lib().oscar_engine_stats(self.h, C.byref(t), C.byref(it))
        return dict(ticks=t.value, cg_iters=it.value)
