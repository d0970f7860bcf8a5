"""CPU FP64 oracle of the 4D phase-space variant (x, y periodic; u, w the
velocities): ctypes wrapper around vp4_oracle.c (built into the same
library as the 1D oracle).

TEST INFRASTRUCTURE ONLY: only the tests, the smoke check and the
benchmark's CPU-baseline leg may import it; the engine never calls it.
"""
from __future__ import annotations

import ctypes as C
import math

import numpy as np

from . import lib as _lib1, _dp, _f64, _check, OracleError

BETA_DEFAULT = 0.5 * (1.0 - math.sqrt(3.0) / 2.0)


class _Params4(C.Structure):
    _fields_ = [("ns", C.c_int32), ("nv", C.c_int32), ("L", C.c_double),
                ("vmax", C.c_double), ("ss", C.c_int32), ("sv", C.c_int32),
                ("G", C.c_double), ("dt", C.c_double), ("n_s", C.c_int32),
                ("beta", C.c_double)]


_ready = False


def lib():
    global _ready
    L = _lib1()
    if not _ready:
        P = C.POINTER
        pd, vp = P(C.c_double), C.c_void_p
        L.or4_create.restype = vp
        L.or4_create.argtypes = [P(_Params4)]
        L.or4_destroy.argtypes = [vp]
        L.or4_destroy.restype = None
        for name, args in [
            ("or4_init_conditions", [vp, pd]),
            ("or4_step", [vp, C.c_int]),
            ("or4_remap", [vp]),
            ("or4_reconstruct_f", [vp, C.c_int, pd]),
            ("or4_density", [vp, pd]),
            ("or4_field", [vp, pd, pd, pd]),
            ("or4_diagnostics", [vp, pd]),
            ("or4_get_elements", [vp, pd]),
            ("or4_set_elements", [vp, pd]),
            ("or4_get_assignment", [vp, C.c_int, P(C.c_int32)]),
            ("or4_spline_fit", [C.c_int, C.c_int, pd, pd]),
            ("or4_inverse_map", [pd, pd, pd, C.c_double, pd]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.or4_time.argtypes = [vp]
        L.or4_time.restype = C.c_double
        for name in ("or4_int15", "or4_spline_eval"):
            fn = getattr(L, name)
            fn.argtypes = [pd, C.c_int, C.c_int, pd]
            fn.restype = C.c_double
        _ready = True
    return L


class Oracle4:
    """One 4D oracle run: ns (space sites per axis), nv (velocity sites per
    axis), L (period), vmax, ss, sv (element spacing in sites), G, dt, n_s,
    beta."""

    def __init__(self, **p):
        self.p = dict(p)
        self.ns, self.nv = int(p["ns"]), int(p["nv"])
        self.ss, self.sv = int(p["ss"]), int(p["sv"])
        self.ms, self.mv = self.ns // self.ss, self.nv // self.sv
        self.E = self.ms ** 2 * self.mv ** 2
        self.shape = (self.nv, self.nv, self.ns, self.ns)  # (w, u, y, x)
        cp = _Params4(self.ns, self.nv, float(p["L"]), float(p["vmax"]),
                      self.ss, self.sv, float(p.get("G", 1.0)),
                      float(p["dt"]), int(p.get("n_s", 0)),
                      float(p.get("beta", BETA_DEFAULT)))
        h = lib().or4_create(C.byref(cp))
        if not h:
            raise OracleError("invalid 4D oracle parameters")
        self.h = C.c_void_p(h)

    def close(self):
        if self.h:
            lib().or4_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def init_conditions(self, f0):
        f0 = _f64(f0).reshape(self.shape)
        _check(lib().or4_init_conditions(self.h, _dp(f0)), "init_conditions")

    def step(self, n: int = 1):
        _check(lib().or4_step(self.h, int(n)), "step")

    def remap(self):
        _check(lib().or4_remap(self.h), "remap")

    def reconstruct_f(self, scheme: int = 0) -> np.ndarray:
        out = np.empty(self.shape)
        _check(lib().or4_reconstruct_f(self.h, int(scheme), _dp(out)),
               "reconstruct_f")
        return out

    def density(self) -> np.ndarray:
        out = np.empty((self.ns, self.ns))
        _check(lib().or4_density(self.h, _dp(out)), "density")
        return out

    def field(self, rho):
        rho = _f64(rho).reshape(self.ns, self.ns)
        ax, ay = np.empty_like(rho), np.empty_like(rho)
        _check(lib().or4_field(self.h, _dp(rho), _dp(ax), _dp(ay)), "field")
        return ax, ay

    def diagnostics(self) -> dict:
        out = np.empty(6)
        _check(lib().or4_diagnostics(self.h, _dp(out)), "diagnostics")
        return dict(zip(("mass", "e_kin", "e_pot", "energy", "entropy", "t"),
                        out.tolist()))

    def get_elements(self) -> np.ndarray:
        out = np.empty((60, self.E))
        _check(lib().or4_get_elements(self.h, _dp(out)), "get_elements")
        return out

    def set_elements(self, el):
        el = _f64(el).reshape(60, self.E)
        _check(lib().or4_set_elements(self.h, _dp(el)), "set_elements")

    def assignment(self, brute: bool = False) -> np.ndarray:
        out = np.empty(self.shape, dtype=np.int32)
        _check(lib().or4_get_assignment(
            self.h, int(brute), out.ctypes.data_as(C.POINTER(C.c_int32))),
            "get_assignment")
        return out

    @property
    def t(self) -> float:
        return lib().or4_time(self.h)


def int15(F, s4) -> float:
    F = _f64(F)
    nv, _, ns, _ = F.shape
    s = _f64(s4)
    return lib().or4_int15(_dp(F), ns, nv, _dp(s))


def spline_fit(F) -> np.ndarray:
    F = _f64(F)
    nv, _, ns, _ = F.shape
    Cc = np.empty_like(F)
    _check(lib().or4_spline_fit(ns, nv, _dp(F), _dp(Cc)), "spline_fit")
    return Cc


def spline_eval(Cc, s4) -> float:
    Cc = _f64(Cc)
    nv, _, ns, _ = Cc.shape
    s = _f64(s4)
    return lib().or4_spline_eval(_dp(Cc), ns, nv, _dp(s))


def inverse_map(el60, Dm, P, L):
    """(dq[4], valid, det) of one element's 4D inverse map at P."""
    out = np.empty(6)
    lib().or4_inverse_map(_dp(_f64(el60)), _dp(_f64(Dm)), _dp(_f64(P)),
                          float(L), _dp(out))
    return out[:4], bool(out[4]), out[5]
