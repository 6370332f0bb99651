"""ctypes wrapper of the FP64 CPU oracle (test infrastructure only)."""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

FIELDS = dict(alpha=0, U=1, p=2, U_vd=3, p_vd=4, U_cr=5, p_cr=6, phi_vd=7, phi_vd_prev=8, phi_cr=9,
              kappa=10, rAU=11, rhs=12, U_sum=13, HbyA=14, nhatf=15)


class _Params(C.Structure):
    _fields_ = [("dim", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("h", C.c_double), ("rho1", C.c_double), ("mu1", C.c_double), ("rho2", C.c_double),
                ("mu2", C.c_double), ("sigma", C.c_double), ("theta_deg", C.c_double),
                ("bc", C.c_int32 * 6), ("u_inlet", C.c_double), ("n_corr", C.c_int32),
                ("pcg_rtol", C.c_double), ("pcg_max_it", C.c_int32), ("mules_iter", C.c_int32)]


class _Stats(C.Structure):
    _fields_ = [("mass", C.c_double), ("max_courant", C.c_double), ("mass_defect", C.c_double),
                ("last_E", C.c_double), ("last_res", C.c_double), ("last_pcg_iters", C.c_int32),
                ("pcg_iters_step", C.c_int32), ("n_fluid", C.c_int32), ("pcg_maxit_hit", C.c_int32),
                ("k_f", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        dp = C.POINTER(C.c_double)
        ip = C.POINTER(C.c_int32)
        L.orc_create.restype = C.c_void_p
        L.orc_create.argtypes = [C.POINTER(_Params), C.POINTER(C.c_uint8), dp]
        L.orc_destroy.argtypes = [C.c_void_p]
        L.orc_field_len.restype = C.c_int64
        L.orc_field_len.argtypes = [C.c_void_p, C.c_int32]
        L.orc_get_field.argtypes = [C.c_void_p, C.c_int32, dp]
        L.orc_set_field.argtypes = [C.c_void_p, C.c_int32, dp]
        L.orc_viscous_step.argtypes = [C.c_void_p, C.c_double]
        L.orc_capillary_relax.argtypes = [C.c_void_p, C.c_double, C.c_int32, C.c_int32, C.c_double, ip, dp]
        L.orc_pressure_solve.argtypes = [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_int32, ip, dp]
        L.orc_dense_solve.argtypes = [C.c_void_p, dp]
        L.orc_get_stats.argtypes = [C.c_void_p, C.POINTER(_Stats)]
        for f in ("orc_dt_brackbill",):
            getattr(L, f).restype = C.c_double
            getattr(L, f).argtypes = [C.c_double] * 4
        L.orc_dt_cfl.restype = C.c_double
        L.orc_dt_cfl.argtypes = [C.c_double] * 2
        L.orc_velocity_from_ca.restype = C.c_double
        L.orc_velocity_from_ca.argtypes = [C.c_double] * 3
        _lib = L
    return _lib


def _dp(a):
    return a.ctypes.data_as(C.POINTER(C.c_double))


class Oracle:
    """One FP64 oracle instance of a case dictionary (see cases.py)."""

    def __init__(self, case, **over):
        c = dict(case)
        c.update(over)
        self.case = c
        p = _Params()
        for k in ("dim", "nx", "ny", "nz", "n_corr", "pcg_max_it"):
            setattr(p, k, int(c[k]))
        for k in ("h", "rho1", "mu1", "rho2", "mu2", "sigma", "theta_deg", "u_inlet", "pcg_rtol"):
            setattr(p, k, float(c[k]))
        for i in range(6):
            p.bc[i] = int(c["bc"][i])
        p.mules_iter = int(c.get("mules_iter", 1))
        self._mask = np.ascontiguousarray(c["mask"], dtype=np.uint8)
        a0 = np.ascontiguousarray(c["alpha0"], dtype=np.float64)
        self.h = lib().orc_create(C.byref(p), self._mask.ctypes.data_as(C.POINTER(C.c_uint8)), _dp(a0))
        if not self.h:
            raise ValueError("oracle rejected the case")
        self.d = int(c["dim"])

    def __del__(self):
        if getattr(self, "h", None):
            lib().orc_destroy(self.h)
            self.h = None

    def get(self, name):
        fid = FIELDS[name]
        n = lib().orc_field_len(self.h, fid)
        out = np.empty(n, dtype=np.float64)
        lib().orc_get_field(self.h, fid, _dp(out))
        return out

    def set(self, name, arr):
        fid = FIELDS[name]
        a = np.ascontiguousarray(arr, dtype=np.float64)
        assert a.size == lib().orc_field_len(self.h, fid)
        rc = lib().orc_set_field(self.h, fid, _dp(a))
        assert rc == 0

    def viscous_step(self, dt_vd):
        return lib().orc_viscous_step(self.h, float(dt_vd))

    def capillary_relax(self, dt_vd, n_sub, max_iters, tol):
        kf = C.c_int32(0)
        E = np.zeros(max(1, max_iters), dtype=np.float64)
        rc = lib().orc_capillary_relax(self.h, float(dt_vd), int(n_sub), int(max_iters), float(tol),
                                        C.byref(kf), _dp(E))
        return rc, kf.value, E[:kf.value].copy()

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
        rc = lib().orc_pressure_solve(self.h, int(which), float(dt), float(rtol), int(max_it),
                                       C.byref(it), C.byref(res))
        return rc, it.value, res.value

    def dense_solve(self):
        out = np.zeros(int(self.case["nx"]) * int(self.case["ny"]) * int(self.case["nz"]))
        rc = lib().orc_dense_solve(self.h, _dp(out))
        assert rc == 0
        return out

    def stats(self):
        s = _Stats()
        lib().orc_get_stats(self.h, C.byref(s))
        return {k: getattr(s, k) for k, _ in _Stats._fields_}


def dt_brackbill(rho1, rho2, h, sigma):
    return lib().orc_dt_brackbill(rho1, rho2, h, sigma)


def dt_cfl(h, u):
    return lib().orc_dt_cfl(h, u)


def velocity_from_ca(ca, mu, sigma):
    return lib().orc_velocity_from_ca(ca, mu, sigma)
