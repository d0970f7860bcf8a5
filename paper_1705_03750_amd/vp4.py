"""Python binding of the 4D phase-space engine (include/vp4.h, libvp4.so):
2D periodic space x 2D velocity.  Argument marshalling only; every step
runs in the library's kernels.  Fails loudly when libvp4.so is missing."""
from __future__ import annotations

import ctypes as C
import math
import os

from . import _live

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB4_PATH = os.path.join(_HERE, "libvp4.so")

FP64, MIXED = 0, 1
BETA_PAPER = 0.5 * (1.0 - math.sqrt(3.0) / 2.0)
EXPORTS = (
    "vp4_footprint", "vp4_create", "vp4_destroy", "vp4_init_conditions",
    "vp4_step", "vp4_remap", "vp4_reconstruct_f", "vp4_density", "vp4_field",
    "vp4_diagnostics", "vp4_get_elements", "vp4_set_elements",
    "vp4_get_assignment", "vp4_prof_begin", "vp4_prof_end", "vp4_sync",
    "vp4_last_error",
)
PROF_KINDS = ("predict", "recon", "field", "kick", "remap_eval", "spline_fit",
              "other")


class Params4(C.Structure):
    _fields_ = [("ns", C.c_int32), ("nv", C.c_int32), ("L", C.c_double),
                ("vmax", C.c_double), ("ss", C.c_int32), ("sv", C.c_int32),
                ("G", C.c_double), ("dt", C.c_double), ("n_s", C.c_int32),
                ("beta", C.c_double), ("precision", C.c_int32)]


class VP4Error(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vp4 error {code}: {msg}")
        self.code = code


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB4_PATH):
            raise RuntimeError(
                f"{LIB4_PATH} is missing: build it with "
                "`python -c 'import __graft_entry__ as g; g.build()'`")
        L = C.CDLL(LIB4_PATH)
        vp, pd = C.c_void_p, C.POINTER(C.c_double)
        sig = {
            "vp4_footprint": [C.POINTER(Params4), C.POINTER(C.c_size_t)],
            "vp4_create": [C.POINTER(Params4), vp, C.c_size_t, vp,
                           C.POINTER(vp)],
            "vp4_destroy": [vp],
            "vp4_init_conditions": [vp, vp],
            "vp4_step": [vp, C.c_int],
            "vp4_remap": [vp],
            "vp4_reconstruct_f": [vp, C.c_int, vp],
            "vp4_density": [vp, vp],
            "vp4_field": [vp, vp, vp, vp],
            "vp4_diagnostics": [vp, pd],
            "vp4_get_elements": [vp, vp],
            "vp4_set_elements": [vp, vp],
            "vp4_get_assignment": [vp, vp],
            "vp4_prof_begin": [vp, C.c_int],
            "vp4_prof_end": [vp, pd, C.POINTER(C.c_int64)],
            "vp4_sync": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.vp4_last_error.argtypes = [vp]
        L.vp4_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def make_params(ns, nv, L, vmax, ss, sv, G=-0.5, dt=0.1, n_s=0,
                beta=BETA_PAPER, precision="fp64") -> Params4:
    prec = {"fp64": FP64, "mixed": MIXED}[precision] \
        if isinstance(precision, str) else int(precision)
    return Params4(int(ns), int(nv), float(L), float(vmax), int(ss), int(sv),
                   float(G), float(dt), int(n_s), float(beta), prec)


class VlasovRun4:
    """One 4D run on a HIP device; keyword parameters follow vp4_params.
    Arrays are torch tensors of shape (nv, nv, ns, ns) = (w, u, y, x)."""

    def __init__(self, device="cuda:0", stream=None, **kw):
        import torch
        self.torch = torch
        self.p = make_params(**kw)
        self.ns, self.nv = self.p.ns, self.p.nv
        self.ms, self.mv = self.ns // self.p.ss, self.nv // self.p.sv
        self.E = self.ms ** 2 * self.mv ** 2
        self.shape = (self.nv, self.nv, self.ns, self.ns)
        self.mixed = self.p.precision == MIXED
        self.device = torch.device(device)
        n = C.c_size_t(0)
        self._chk(lib().vp4_footprint(C.byref(self.p), C.byref(n)), None)
        self.ws = torch.empty(int(n.value), dtype=torch.uint8,
                              device=self.device)
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._chk(lib().vp4_create(C.byref(self.p),
                                   C.c_void_p(self.ws.data_ptr()),
                                   int(n.value),
                                   C.c_void_p(self.stream.cuda_stream),
                                   C.byref(h)), None)
        self.h = h
        self._keep = []
        _live.add(self)

    def _chk(self, rc, h):
        if rc != 0:
            msg = lib().vp4_last_error(h)
            raise VP4Error(rc, (msg or b"").decode())

    def _dev(self, x, dtype):
        t = self.torch.as_tensor(x, device=self.device, dtype=dtype)
        return t.contiguous()

    def init_conditions(self, f0):
        t = self._dev(f0, self.torch.float64).reshape(self.shape)
        self._keep = [t]
        self._chk(lib().vp4_init_conditions(self.h, C.c_void_p(t.data_ptr())),
                  self.h)

    def step(self, n=1):
        self._chk(lib().vp4_step(self.h, int(n)), self.h)

    def remap(self):
        self._chk(lib().vp4_remap(self.h), self.h)

    def reconstruct_f(self, scheme=0):
        dt = self.torch.float32 if self.mixed else self.torch.float64
        out = self.torch.empty(self.shape, dtype=dt, device=self.device)
        self._chk(lib().vp4_reconstruct_f(self.h, int(scheme),
                                          C.c_void_p(out.data_ptr())), self.h)
        return out

    def density(self):
        out = self.torch.empty((self.ns, self.ns), dtype=self.torch.float64,
                               device=self.device)
        self._chk(lib().vp4_density(self.h, C.c_void_p(out.data_ptr())),
                  self.h)
        return out

    def field(self, rho):
        r = self._dev(rho, self.torch.float64).reshape(self.ns, self.ns)
        ax = self.torch.empty_like(r)
        ay = self.torch.empty_like(r)
        self._keep = [r]
        self._chk(lib().vp4_field(self.h, C.c_void_p(r.data_ptr()),
                                  C.c_void_p(ax.data_ptr()),
                                  C.c_void_p(ay.data_ptr())), self.h)
        return ax, ay

    def diagnostics(self) -> dict:
        out = (C.c_double * 6)()
        self._chk(lib().vp4_diagnostics(self.h, out), self.h)
        return dict(zip(("mass", "e_kin", "e_pot", "energy", "entropy", "t"),
                        list(out)))

    def get_elements(self):
        out = self.torch.empty((60, self.E), dtype=self.torch.float64,
                               device=self.device)
        self._chk(lib().vp4_get_elements(self.h, C.c_void_p(out.data_ptr())),
                  self.h)
        return out

    def set_elements(self, el):
        t = self._dev(el, self.torch.float64).reshape(60, self.E)
        self._keep = [t]
        self._chk(lib().vp4_set_elements(self.h, C.c_void_p(t.data_ptr())),
                  self.h)

    def assignment(self):
        out = self.torch.empty(self.shape, dtype=self.torch.int32,
                               device=self.device)
        self._chk(lib().vp4_get_assignment(self.h, C.c_void_p(out.data_ptr())),
                  self.h)
        return out

    def prof_begin(self, max_launches):
        self._chk(lib().vp4_prof_begin(self.h, int(max_launches)), self.h)

    def prof_end(self):
        ms = (C.c_double * 7)()
        n = (C.c_int64 * 7)()
        self._chk(lib().vp4_prof_end(self.h, ms, n), self.h)
        return {k: (ms[i], n[i]) for i, k in enumerate(PROF_KINDS)}

    def sync(self):
        self._chk(lib().vp4_sync(self.h), self.h)

    def close(self):
        if getattr(self, "h", None):
            lib().vp4_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
