"""CPU FP64 oracle of the metric semi-Lagrangian Vlasov-Poisson method
(Colombi & Alard, arXiv:1705.03750): ctypes wrapper around vp_oracle.c.

TEST INFRASTRUCTURE ONLY.  Only the tests, the smoke check and the
benchmark's CPU-baseline leg may import this package.  It shares no code
with the HIP engine and the engine never calls it.

`build()` compiles the C source with gcc (-O2 -ffp-contract=off, optional
OpenMP); `Oracle(params)` wraps one run.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "vp_oracle.c")
_SRC4 = os.path.join(_HERE, "vp4_oracle.c")
_OUTDIR = os.path.join(_HERE, "_build")
_LIB_PATH = os.path.join(_OUTDIR, "liboracle.so")

FORCE_SELF = 0
FORCE_EXTERNAL = 1
BC_ISOLATED = 0
BC_PERIODIC = 1
SCHEME_TRANSPORT = 0
SCHEME_REMAP = 1
BETA_DEFAULT = 0.5 * (1.0 - math.sqrt(3.0) / 2.0)


def build(verbose: bool = False) -> str:
    """Compile the oracle into oracle/_build/liboracle.so (always rebuilds)."""
    os.makedirs(_OUTDIR, exist_ok=True)
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
           "-fPIC", "-shared", "-fopenmp", "-Wall", "-o", tmp, _SRC, _SRC4,
           "-lm"]
    res = subprocess.run(cmd, capture_output=True, text=True)
    if res.returncode != 0:
        raise RuntimeError("oracle build failed:\n" + res.stderr)
    if verbose and res.stderr:
        print(res.stderr)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nv", C.c_int32),
                ("x_min", C.c_double), ("x_max", C.c_double),
                ("v_min", C.c_double), ("v_max", C.c_double),
                ("sx", C.c_int32), ("sv", C.c_int32),
                ("G", C.c_double), ("dt", C.c_double),
                ("n_s", C.c_int32), ("beta", C.c_double),
                ("force_mode", C.c_int32),
                ("ext_a0", C.c_double), ("ext_a1", C.c_double),
                ("ext_a2", C.c_double),
                ("emap_max", C.c_double), ("emap_every", C.c_int32),
                ("cdyn", C.c_double), ("bc", C.c_int32)]


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        L = C.CDLL(_LIB_PATH)
        P = C.POINTER
        d, i32, i64, vp = C.c_double, C.c_int32, C.c_int64, C.c_void_p
        pd = P(C.c_double)
        L.or_create.restype = vp
        L.or_create.argtypes = [P(_Params)]
        L.or_destroy.argtypes = [vp]
        L.or_destroy.restype = None
        for name, args in [
            ("or_init_conditions", [vp, pd]),
            ("or_step", [vp, C.c_int]),
            ("or_remap", [vp]),
            ("or_reconstruct_f", [vp, C.c_int, pd]),
            ("or_reconstruct_sites", [vp, C.c_int, i64, P(i64), pd]),
            ("or_density", [vp, pd]),
            ("or_remap_position", [vp, i64, pd, pd]),
            ("or_poisson", [vp, pd, pd, pd, pd]),
            ("or_diagnostics", [vp, pd]),
            ("or_emap", [vp, pd]),
            ("or_get_elements", [vp, pd]),
            ("or_set_elements", [vp, pd]),
            ("or_get_assignment", [vp, C.c_int, P(i32)]),
            ("or_get_F", [vp, pd]),
            ("or_get_coeffs", [vp, pd]),
            ("or_spline_fit", [C.c_int, C.c_int, pd, pd]),
            ("or_spline_fit_periodic", [C.c_int, C.c_int, pd, pd]),
            ("or_inverse_map", [pd, d, d, d, d, pd]),
        ]:
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.or_set_threads.argtypes = [C.c_int]
        L.or_set_threads.restype = C.c_int
        L.or_time.argtypes = [vp]
        L.or_time.restype = d
        L.or_dt.argtypes = [vp]
        L.or_dt.restype = d
        L.or_stepcount.argtypes = [vp]
        L.or_stepcount.restype = i64
        for name in ("or_int1", "or_int1_periodic", "or_spline_eval",
                     "or_spline_eval_periodic"):
            fn = getattr(L, name)
            fn.argtypes = [pd, C.c_int, C.c_int, d, d]
            fn.restype = d
        L.or_W.argtypes = [d]
        L.or_W.restype = d
        L.or_tsc.argtypes = [pd, C.c_int, d]
        L.or_tsc.restype = d
        _lib = L
    return _lib


def _dp(a: np.ndarray):
    return a.ctypes.data_as(C.POINTER(C.c_double))


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def set_threads(n: int) -> int:
    return lib().or_set_threads(int(n))


class Oracle:
    """One oracle run.  `params` uses the engine's field names (nx, nv,
    x_min..v_max, sx, sv, G, dt, n_s, beta, force_mode, ext_a0..ext_a2,
    emap_max, emap_every, c_dyn, bc)."""

    def __init__(self, **p):
        self.p = dict(p)
        self.nx = int(p["nx"])
        self.nv = int(p.get("nv") or self.nx)
        self.sx = int(p["sx"])
        self.sv = int(p.get("sv") or self.sx)
        self.mx, self.mv = self.nx // self.sx, self.nv // self.sv
        self.E = self.mx * self.mv
        ext = p.get("ext", (0.0, 0.0, 0.0))
        cp = _Params(self.nx, self.nv, p.get("x_min", -1.0),
                     p.get("x_max", 1.0), p.get("v_min", -1.0),
                     p.get("v_max", 1.0), self.sx, self.sv, p.get("G", 1.0),
                     p["dt"], int(p.get("n_s", 0)),
                     p.get("beta", BETA_DEFAULT),
                     int(p.get("force_mode", FORCE_SELF)),
                     ext[0], ext[1], ext[2],
                     float(p.get("emap_max", 0.0)),
                     int(p.get("emap_every", 0)),
                     float(p.get("c_dyn", 0.0)),
                     int(p.get("bc", BC_ISOLATED)))
        self._p = cp
        h = lib().or_create(C.byref(cp))
        if not h:
            raise OracleError("invalid oracle parameters")
        self.h = C.c_void_p(h)

    def close(self):
        if self.h:
            lib().or_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # --- calls -----------------------------------------------------------
    def init_conditions(self, f0):
        f0 = _f64(f0).reshape(self.nv, self.nx)
        _check(lib().or_init_conditions(self.h, _dp(f0)), "init_conditions")

    def step(self, n: int = 1):
        _check(lib().or_step(self.h, int(n)), "step")

    def remap(self):
        _check(lib().or_remap(self.h), "remap")

    def reconstruct_f(self, scheme: int = SCHEME_TRANSPORT) -> np.ndarray:
        out = np.empty((self.nv, self.nx))
        _check(lib().or_reconstruct_f(self.h, int(scheme), _dp(out)),
               "reconstruct_f")
        return out

    def reconstruct_sites(self, sites, scheme: int = SCHEME_TRANSPORT):
        s = np.ascontiguousarray(sites, dtype=np.int64)
        out = np.empty(s.shape[0])
        _check(lib().or_reconstruct_sites(
            self.h, int(scheme), s.shape[0],
            s.ctypes.data_as(C.POINTER(C.c_int64)), _dp(out)),
            "reconstruct_sites")
        return out

    def remap_position(self, P) -> np.ndarray:
        """Blended Lagrangian position Q_r(P) of eq. (interpol) at arbitrary
        phase-space points P (shape (n, 2)); NaN where no element is valid."""
        P = _f64(P).reshape(-1, 2)
        out = np.empty_like(P)
        _check(lib().or_remap_position(self.h, P.shape[0], _dp(P), _dp(out)),
               "remap_position")
        return out

    def density(self) -> np.ndarray:
        out = np.empty(self.nx)
        _check(lib().or_density(self.h, _dp(out)), "density")
        return out

    def poisson(self, rho):
        rho = _f64(rho)
        a, da, d2a = (np.empty(self.nx) for _ in range(3))
        _check(lib().or_poisson(self.h, _dp(rho), _dp(a), _dp(da), _dp(d2a)),
               "poisson")
        return a, da, d2a

    def diagnostics(self) -> dict:
        out = np.empty(9)
        _check(lib().or_diagnostics(self.h, _dp(out)), "diagnostics")
        keys = ("mass", "e_kin", "e_pot", "energy", "entropy", "max_det_dev",
                "t", "l1", "l2")
        return dict(zip(keys, out.tolist()))

    def emap(self) -> float:
        """E_map of the current elements, in element-spacing units."""
        out = C.c_double(0.0)
        _check(lib().or_emap(self.h, C.byref(out)), "emap")
        return out.value

    def get_elements(self) -> np.ndarray:
        out = np.empty((12, self.E))
        _check(lib().or_get_elements(self.h, _dp(out)), "get_elements")
        return out

    def set_elements(self, el):
        el = _f64(el).reshape(12, self.E)
        _check(lib().or_set_elements(self.h, _dp(el)), "set_elements")

    def assignment(self, brute: bool = False) -> np.ndarray:
        out = np.empty((self.nv, self.nx), dtype=np.int32)
        _check(lib().or_get_assignment(
            self.h, int(brute), out.ctypes.data_as(C.POINTER(C.c_int32))),
            "get_assignment")
        return out

    def F(self) -> np.ndarray:
        out = np.empty((self.nv, self.nx))
        _check(lib().or_get_F(self.h, _dp(out)), "get_F")
        return out

    def coeffs(self) -> np.ndarray:
        out = np.empty((self.nv, self.nx))
        _check(lib().or_get_coeffs(self.h, _dp(out)), "get_coeffs")
        return out

    @property
    def t(self) -> float:
        return lib().or_time(self.h)

    @property
    def dt(self) -> float:
        """The step size the next step takes (the nominal dt unless
        c_dyn > 0)."""
        return lib().or_dt(self.h)

    @property
    def stepcount(self) -> int:
        return lib().or_stepcount(self.h)


# --- primitives -----------------------------------------------------------
def int1(F, sx: float, sv: float, periodic: bool = False) -> float:
    F = _f64(F)
    nv, nx = F.shape
    fn = lib().or_int1_periodic if periodic else lib().or_int1
    return fn(_dp(F), nx, nv, float(sx), float(sv))


def W(x: float) -> float:
    return lib().or_W(float(x))


def spline_fit(F, periodic: bool = False) -> np.ndarray:
    F = _f64(F)
    nv, nx = F.shape
    Cc = np.empty_like(F)
    fn = lib().or_spline_fit_periodic if periodic else lib().or_spline_fit
    _check(fn(nx, nv, _dp(F), _dp(Cc)), "spline_fit")
    return Cc


def spline_eval(Cc, sx: float, sv: float, periodic: bool = False) -> float:
    Cc = _f64(Cc)
    nv, nx = Cc.shape
    fn = lib().or_spline_eval_periodic if periodic else lib().or_spline_eval
    return fn(_dp(Cc), nx, nv, float(sx), float(sv))


def inverse_map(el12, dxm, dvm, xP, vP):
    """Returns (dqx, dqv, valid, det) of one element's inverse map at P."""
    el = _f64(el12)
    out = np.empty(4)
    lib().or_inverse_map(_dp(el), float(dxm), float(dvm), float(xP),
                         float(vP), _dp(out))
    return out[0], out[1], bool(out[2]), out[3]


def tsc(g, u: float) -> float:
    g = _f64(g)
    return lib().or_tsc(_dp(g), g.shape[0], float(u))
