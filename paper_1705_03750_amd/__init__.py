"""MI355X engine for the metric semi-Lagrangian Vlasov-Poisson method of
Colombi & Alard (arXiv:1705.03750).

Thin Python binding of the C ABI in include/vp.h (libvp.so, HIP kernels for
gfx950).  It only marshals arguments: every step of the method runs in the
library's kernels.  PyTorch provides the device workspace and the stream.
The binding fails loudly when libvp.so is missing; there is no fallback.
"""
from __future__ import annotations

import atexit
import ctypes as C
import weakref
import math
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libvp.so")

OK, EINVAL, ENOMEM, EDEVICE, ESTATE, ENUMERIC = 0, -1, -2, -3, -4, -5
FP64, MIXED = 0, 1
FORCE_SELF, FORCE_EXTERNAL = 0, 1
BC_ISOLATED, BC_PERIODIC = 0, 1
SCHEME_TRANSPORT, SCHEME_REMAP = 0, 1
BETA_PAPER = 0.5 * (1.0 - math.sqrt(3.0) / 2.0)

EXPORTS = (
    "vp_footprint", "vp_create", "vp_destroy", "vp_init_conditions",
    "vp_step", "vp_remap", "vp_reconstruct_f", "vp_density", "vp_poisson",
    "vp_poisson_static", "vp_diagnostics", "vp_get_elements", "vp_set_elements",
    "vp_get_assignment", "vp_time", "vp_sync", "vp_last_error",
    "vp_prof_begin", "vp_prof_end", "vp_server_footprint", "vp_server_create",
    "vp_server_run", "vp_server_destroy", "vp_server_last_error",
)
PROF_KINDS = ("predict", "recon", "field", "kick", "remap_eval", "spline_fit",
              "reset", "other")


class Params(C.Structure):
    _fields_ = [("nx", C.c_int32), ("nv", C.c_int32),
                ("x_min", C.c_double), ("x_max", C.c_double),
                ("v_min", C.c_double), ("v_max", C.c_double),
                ("sx", C.c_int32), ("sv", C.c_int32),
                ("G", C.c_double), ("dt", C.c_double),
                ("n_s", C.c_int32), ("beta", C.c_double),
                ("force_mode", C.c_int32),
                ("ext_a0", C.c_double), ("ext_a1", C.c_double),
                ("ext_a2", C.c_double), ("precision", C.c_int32),
                ("emap_max", C.c_double), ("emap_every", C.c_int32),
                ("c_dyn", C.c_double), ("bc", C.c_int32)]


class Diag(C.Structure):
    _fields_ = [("mass", C.c_double), ("e_kin", C.c_double),
                ("e_pot", C.c_double), ("energy", C.c_double),
                ("entropy", C.c_double), ("max_det_dev", C.c_double),
                ("t", C.c_double), ("step", C.c_int64),
                ("overflow_blocks", C.c_int64), ("emap", C.c_double),
                ("dt", C.c_double), ("l1", C.c_double), ("l2", C.c_double)]


class Request(C.Structure):
    _fields_ = [("params", Params), ("f0_dev", C.c_void_p),
                ("f_out_dev", C.c_void_p), ("nsteps", C.c_int32),
                ("pad", C.c_int32), ("tag", C.c_int64),
                ("arrival_s", C.c_double)]


class RequestResult(C.Structure):
    _fields_ = [("tag", C.c_int64), ("arrival_s", C.c_double),
                ("admit_s", C.c_double), ("done_s", C.c_double),
                ("status", C.c_int32), ("pad", C.c_int32)]


class ServerStats(C.Structure):
    _fields_ = [("wall_s", C.c_double), ("gpu_busy_s", C.c_double),
                ("ticks", C.c_int64), ("site_updates", C.c_int64),
                ("admitted", C.c_int64), ("completed", C.c_int64),
                ("max_active", C.c_int32), ("graph_replay", C.c_int32)]


class VPError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"vp error {code}: {msg}")
        self.code = code


_lib = None

# Every live run and server, closed by an exit handler: the library's HIP
# streams, events and pinned buffers are released while the runtime is
# still whole, not by finalisers during interpreter teardown.
_live = weakref.WeakSet()


def _close_all():
    for obj in list(_live):
        try:
            obj.close()
        except Exception:
            pass


atexit.register(_close_all)


def lib():
    """Load libvp.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"{LIB_PATH} is missing: build it with "
                "paper_1705_03750_amd.build.build() (hipcc, gfx950)")
        L = C.CDLL(LIB_PATH)
        vp, pd, pp = C.c_void_p, C.POINTER(C.c_double), C.POINTER(Params)
        sig = {
            "vp_footprint": [pp, C.POINTER(C.c_size_t)],
            "vp_create": [pp, vp, C.c_size_t, vp, C.POINTER(vp)],
            "vp_destroy": [vp],
            "vp_init_conditions": [vp, vp, C.c_int],
            "vp_step": [vp, C.c_int],
            "vp_remap": [vp],
            "vp_reconstruct_f": [vp, C.c_int, vp],
            "vp_density": [vp, vp],
            "vp_poisson": [vp, vp, vp, vp, vp],
            "vp_poisson_static": [pp, vp, vp, vp, vp, vp],
            "vp_diagnostics": [vp, C.POINTER(Diag)],
            "vp_get_elements": [vp, vp],
            "vp_set_elements": [vp, vp],
            "vp_get_assignment": [vp, vp],
            "vp_time": [vp, pd, C.POINTER(C.c_int64)],
            "vp_sync": [vp],
            "vp_prof_begin": [vp, C.c_int],
            "vp_prof_end": [vp, pd, C.POINTER(C.c_int64)],
            "vp_server_footprint": [C.c_int, C.POINTER(C.c_size_t)],
            "vp_server_create": [C.c_int, C.c_int, vp, C.c_size_t, vp,
                                 C.POINTER(vp)],
            "vp_server_run": [vp, C.POINTER(Request), C.c_int,
                              C.POINTER(RequestResult),
                              C.POINTER(ServerStats)],
            "vp_server_destroy": [vp],
        }
        for name, args in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = C.c_int
        L.vp_last_error.argtypes = [vp]
        L.vp_last_error.restype = C.c_char_p
        L.vp_server_last_error.argtypes = [vp]
        L.vp_server_last_error.restype = C.c_char_p
        _lib = L
    return _lib


def make_params(nx, nv=None, x_min=-1.0, x_max=1.0, v_min=-1.0, v_max=1.0,
                sx=8, sv=None, G=1.0, dt=1e-3, n_s=0, beta=BETA_PAPER,
                force_mode=FORCE_SELF, ext=(0.0, 0.0, 0.0),
                precision="fp64", emap_max=0.0, emap_every=0,
                c_dyn=0.0, bc=0) -> Params:
    prec = {"fp64": FP64, "mixed": MIXED}[precision] \
        if isinstance(precision, str) else int(precision)
    nv = nx if nv is None else nv
    sv = sx if sv is None else sv
    return Params(int(nx), int(nv), float(x_min), float(x_max), float(v_min),
                  float(v_max), int(sx), int(sv), float(G), float(dt),
                  int(n_s), float(beta), int(force_mode), float(ext[0]),
                  float(ext[1]), float(ext[2]), prec, float(emap_max),
                  int(emap_every), float(c_dyn), int(bc))


def footprint(**kw) -> int:
    p = make_params(**kw)
    n = C.c_size_t(0)
    rc = lib().vp_footprint(C.byref(p), C.byref(n))
    if rc:
        raise VPError(rc, "invalid parameters")
    return int(n.value)


def poisson_static(rho, stream=None, **kw):
    """a, a', a'' of a density (nx float64 values on a HIP device) through
    vp_poisson_static: no run context, no workspace, nothing allocated by
    the library (outputs are new torch tensors here).  Keyword parameters as
    VlasovRun (nx taken from rho)."""
    import torch
    r = rho if isinstance(rho, torch.Tensor) else torch.as_tensor(rho)
    if r.device.type != "cuda":
        raise ValueError("rho must be a device tensor")
    r = r.to(torch.float64).contiguous()
    kw = dict(kw)
    kw["nx"] = int(r.numel())
    kw.setdefault("sx", 4 if kw["nx"] % 8 else 8)
    p = make_params(**kw)
    outs = [torch.empty_like(r) for _ in range(3)]
    st = stream if stream is not None else torch.cuda.current_stream(r.device)
    rc = lib().vp_poisson_static(C.byref(p), C.c_void_p(r.data_ptr()),
                                 *[C.c_void_p(o.data_ptr()) for o in outs],
                                 C.c_void_p(st.cuda_stream))
    if rc:
        raise VPError(rc, (lib().vp_last_error(None) or b"").decode())
    return tuple(outs)


class VlasovRun:
    """One run of the engine on a CUDA (HIP) device.

    Keyword parameters follow vp_params (nx, nv, x_min..v_max, sx, sv, G,
    dt, n_s, beta, force_mode, ext=(a0, a1, a2), precision='fp64'|'mixed',
    emap_max, emap_every, c_dyn, bc).
    The workspace is one torch uint8 tensor; work is enqueued on the current
    torch stream of `device` (or `stream`, a torch.cuda.Stream)."""

    def __init__(self, device="cuda:0", stream=None, workspace=None, **kw):
        import torch
        self.torch = torch
        self.p = make_params(**kw)
        self.nx, self.nv = self.p.nx, self.p.nv
        self.mx, self.mv = self.nx // self.p.sx, self.nv // self.p.sv
        self.E = self.mx * self.mv
        self.mixed = self.p.precision == MIXED
        self.fdtype = torch.float32 if self.mixed else torch.float64
        self.device = torch.device(device)
        n = C.c_size_t(0)
        self._chk(lib().vp_footprint(C.byref(self.p), C.byref(n)), None)
        self.bytes = int(n.value)
        if workspace is None:
            workspace = torch.empty(self.bytes, dtype=torch.uint8,
                                    device=self.device)
        self.ws = workspace
        self.stream = stream or torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        self._chk(lib().vp_create(C.byref(self.p), C.c_void_p(self.ws.data_ptr()),
                                  self.bytes, C.c_void_p(self.stream.cuda_stream),
                                  C.byref(h)), None)
        self.h = h
        self._keep = []
        _live.add(self)

    # ----------------------------------------------------------------
    def _chk(self, rc, h):
        if rc != 0:
            msg = lib().vp_last_error(h if h is not None else None)
            raise VPError(rc, (msg or b"").decode())

    def _t(self, x, dtype):
        t = self.torch
        if not isinstance(x, t.Tensor):
            x = t.as_tensor(np.ascontiguousarray(x))
        return x.to(device=self.device, dtype=dtype).contiguous()

    def close(self):
        if getattr(self, "h", None):
            lib().vp_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # ---------------------------------------------------------- calls
    def init_conditions(self, f0):
        f = self._t(f0, self.torch.float64).reshape(self.nv, self.nx)
        self._keep = [f]
        self._chk(lib().vp_init_conditions(self.h, C.c_void_p(f.data_ptr()), 1),
                  self.h)

    def step(self, n: int = 1):
        self._chk(lib().vp_step(self.h, int(n)), self.h)

    def remap(self):
        self._chk(lib().vp_remap(self.h), self.h)

    def reconstruct_f(self, scheme: int = SCHEME_TRANSPORT, out=None):
        if out is None:
            out = self.torch.empty((self.nv, self.nx), dtype=self.fdtype,
                                   device=self.device)
        self._chk(lib().vp_reconstruct_f(self.h, int(scheme),
                                         C.c_void_p(out.data_ptr())), self.h)
        return out

    def density(self, out=None):
        if out is None:
            out = self.torch.empty(self.nx, dtype=self.torch.float64,
                                   device=self.device)
        self._chk(lib().vp_density(self.h, C.c_void_p(out.data_ptr())), self.h)
        return out

    def poisson(self, rho):
        r = self._t(rho, self.torch.float64)
        outs = [self.torch.empty(self.nx, dtype=self.torch.float64,
                                 device=self.device) for _ in range(3)]
        self._keep = [r]
        self._chk(lib().vp_poisson(self.h, C.c_void_p(r.data_ptr()),
                                   *[C.c_void_p(o.data_ptr()) for o in outs]),
                  self.h)
        return tuple(outs)

    def diagnostics(self) -> dict:
        d = Diag()
        self._chk(lib().vp_diagnostics(self.h, C.byref(d)), self.h)
        return {k: getattr(d, k) for k, _ in Diag._fields_}

    def get_elements(self):
        out = self.torch.empty((12, self.E), dtype=self.torch.float64,
                               device=self.device)
        self._chk(lib().vp_get_elements(self.h, C.c_void_p(out.data_ptr())),
                  self.h)
        return out

    def set_elements(self, el):
        e = self._t(el, self.torch.float64).reshape(12, self.E)
        self._keep = [e]
        self._chk(lib().vp_set_elements(self.h, C.c_void_p(e.data_ptr())),
                  self.h)

    def assignment(self):
        out = self.torch.empty((self.nv, self.nx), dtype=self.torch.int32,
                               device=self.device)
        self._chk(lib().vp_get_assignment(self.h, C.c_void_p(out.data_ptr())),
                  self.h)
        return out

    def time(self):
        t = C.c_double(0.0)
        s = C.c_int64(0)
        self._chk(lib().vp_time(self.h, C.byref(t), C.byref(s)), self.h)
        return t.value, s.value

    def prof_begin(self, max_launches: int):
        self._chk(lib().vp_prof_begin(self.h, int(max_launches)), self.h)

    def prof_end(self) -> dict:
        ms = (C.c_double * 8)()
        n = (C.c_int64 * 8)()
        self._chk(lib().vp_prof_end(self.h, ms, n), self.h)
        return {k: (ms[i], n[i]) for i, k in enumerate(PROF_KINDS)}

    def sync(self):
        self._chk(lib().vp_sync(self.h), self.h)
        self._keep = []


class Server:
    """Continuous-batching server (vp_server_* in include/vp.h) over one
    device pool (a torch uint8 tensor of pool_bytes)."""

    def __init__(self, precision="mixed", max_active=64, pool_bytes=1 << 31,
                 device="cuda:0"):
        import torch
        self.torch = torch
        self.precision = {"fp64": FP64, "mixed": MIXED}[precision]
        self.device = torch.device(device)
        self.pool = torch.empty(int(pool_bytes), dtype=torch.uint8,
                                device=self.device)
        stream = torch.cuda.current_stream(self.device)
        h = C.c_void_p()
        rc = lib().vp_server_create(self.precision, int(max_active),
                                    C.c_void_p(self.pool.data_ptr()),
                                    int(pool_bytes),
                                    C.c_void_p(stream.cuda_stream), C.byref(h))
        if rc:
            raise VPError(rc, lib().vp_server_last_error(None).decode())
        self.h = h
        _live.add(self)

    def run(self, requests):
        """requests: list of dicts with params (make_params kwargs), f0
        (device float64 tensor), out (device tensor), nsteps, tag, arrival_s
        (ascending).  Returns (results list of dicts, stats dict)."""
        n = len(requests)
        arr = (Request * max(n, 1))()
        for i, r in enumerate(requests):
            arr[i].params = make_params(**r["params"])
            arr[i].f0_dev = r["f0"].data_ptr()
            arr[i].f_out_dev = r["out"].data_ptr()
            arr[i].nsteps = int(r["nsteps"])
            arr[i].tag = int(r.get("tag", i))
            arr[i].arrival_s = float(r.get("arrival_s", 0.0))
        res = (RequestResult * max(n, 1))()
        st = ServerStats()
        rc = lib().vp_server_run(self.h, arr, n, res, C.byref(st))
        if rc:
            raise VPError(rc, lib().vp_server_last_error(self.h).decode())
        out = [{k: getattr(res[i], k) for k, _ in RequestResult._fields_
                if k != "pad"} for i in range(n)]
        stats = {k: getattr(st, k) for k, _ in ServerStats._fields_}
        return out, stats

    def close(self):
        if getattr(self, "h", None):
            lib().vp_server_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
