"""Seeded synthetic initial conditions and run parameters for the 1D
self-gravitating Vlasov-Poisson workloads.

This module is shared by the CPU oracle's tests, the GPU tests and the
benchmark.  It holds none of the method's arithmetic: it only samples an
initial phase-space density f0 on the cell-centred site grid and states the
run parameters (grid, element stride, time step, remap cadence).

Grid convention: site (i, j) sits at x_i = x_min + (i + 1/2) dx,
v_j = v_min + (j + 1/2) dv; arrays are (nv, nx), row-major, v rows, x
fastest.  Every generator zeroes the outermost ring of sites (f = 0 at the
box edges) and rescales the grid mass dx dv sum(f) to the requested total.

The workloads stand in for the paper's initial conditions (section 3.2): a
single Gaussian like its Gaussian run, the thermal-equilibrium sheet of its
stationary run, and seeded sums of Gaussian halos in place of its random set
of stationary clouds, whose exact recipe is not given in the paper.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

__all__ = [
    "RunConfig", "site_coords", "finish", "gaussian_blob", "halo_sum",
    "spitzer_sheet", "two_stream", "landau4", "config", "CONFIGS", "serving_requests",
]


@dataclasses.dataclass
class RunConfig:
    """Run parameters for one workload (box, grid, elements, time)."""
    name: str
    n: int                 # sites per axis (square grids)
    s: int                 # element stride in sites
    dt: float
    steps: int
    n_s: int               # steps between remaps (0 = never)
    G: float = 1.0
    box: tuple = (-1.0, 1.0, -1.0, 1.0)
    seed: int = 0
    bc: int = 0            # 1: x periodic (plasma / periodic gravity)

    def params(self, precision: str = "fp64") -> dict:
        x0, x1, v0, v1 = self.box
        return dict(nx=self.n, nv=self.n, x_min=x0, x_max=x1, v_min=v0,
                    v_max=v1, sx=self.s, sv=self.s, G=self.G, dt=self.dt,
                    n_s=self.n_s, precision=precision, bc=self.bc)


def site_coords(n: int, lo: float, hi: float) -> np.ndarray:
    """Cell-centred site coordinates lo + (i + 1/2) (hi - lo) / n."""
    d = (hi - lo) / n
    return lo + (np.arange(n, dtype=np.float64) + 0.5) * d


def finish(f: np.ndarray, box, mass: float | None = 1.0,
           floor_rel: float = 1e-30) -> np.ndarray:
    """Zero the outer ring, flush values below floor_rel * max to zero and
    rescale the grid mass dx dv sum(f) to `mass` (None keeps the scale)."""
    f = np.array(f, dtype=np.float64, copy=True)
    f[0, :] = 0.0
    f[-1, :] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    fmax = float(np.abs(f).max()) if f.size else 0.0
    if fmax > 0.0:
        f[np.abs(f) < floor_rel * fmax] = 0.0
    if mass is not None:
        nv, nx = f.shape
        x0, x1, v0, v1 = box
        dx = (x1 - x0) / nx
        dv = (v1 - v0) / nv
        m = dx * dv * float(f.sum())
        if m > 0.0:
            f *= mass / m
    return np.ascontiguousarray(f)


def _grids(nx: int, nv: int, box):
    x0, x1, v0, v1 = box
    x = site_coords(nx, x0, x1)
    v = site_coords(nv, v0, v1)
    return x[None, :], v[:, None]


def gaussian_blob(nx: int, nv: int, box, xc: float, vc: float, sx: float,
                  sv: float, amplitude: float = 1.0) -> np.ndarray:
    """amplitude * exp(-(x-xc)^2/(2 sx^2) - (v-vc)^2/(2 sv^2)) on the sites."""
    X, V = _grids(nx, nv, box)
    return amplitude * np.exp(-0.5 * ((X - xc) / sx) ** 2
                              - 0.5 * ((V - vc) / sv) ** 2)


def _unit_gaussian(nx, nv, box, xc, vc, sx, sv):
    # normalised to unit continuum mass
    return gaussian_blob(nx, nv, box, xc, vc, sx, sv,
                         1.0 / (2.0 * math.pi * sx * sv))


def halo_sum(nx: int, nv: int, box, rng: np.random.Generator, k: int,
             mass: float = 1.0) -> np.ndarray:
    """Sum of k Gaussian halos: centres x_c ~ U(-0.5, 0.5), v_c ~ U(-0.3, 0.3),
    dispersions ~ U(0.05, 0.15), masses from a flat Dirichlet draw."""
    xc = rng.uniform(-0.5, 0.5, size=k)
    vc = rng.uniform(-0.3, 0.3, size=k)
    sx = rng.uniform(0.05, 0.15, size=k)
    sv = rng.uniform(0.05, 0.15, size=k)
    w = rng.dirichlet(np.ones(k)) * mass
    f = np.zeros((nv, nx))
    for a in range(k):
        f += w[a] * _unit_gaussian(nx, nv, box, xc[a], vc[a], sx[a], sv[a])
    return f


def spitzer_sheet(nx: int, nv: int, box, rho_s: float = 4.0,
                  sigma_s: float = 0.2, G: float = 1.0) -> np.ndarray:
    """Thermal-equilibrium (isothermal) sheet of section 3.2:
    rho_s / cosh^2(x / x0) * exp(-v^2 / (2 sigma_s^2)) with
    1/x0 = sqrt(sqrt(2 pi) G rho_s / sigma_s), stationary when the force
    is a = G (M_right - M_left)."""
    X, V = _grids(nx, nv, box)
    k = math.sqrt(math.sqrt(2.0 * math.pi) * G * rho_s / sigma_s)
    return rho_s / np.cosh(k * X) ** 2 * np.exp(-0.5 * (V / sigma_s) ** 2)


def _sech2_sheet(nx, nv, box, x0, sigma_v):
    X, V = _grids(nx, nv, box)
    return 1.0 / np.cosh(X / x0) ** 2 * np.exp(-0.5 * (V / sigma_v) ** 2)


# ---------------------------------------------------------------------------
# The five workloads.  Sizes and recipes follow the benchmark configurations;
# seeds are fixed per workload.
CONFIGS = {
    "c1_gaussian_256": RunConfig("c1_gaussian_256", n=256, s=4, dt=1e-3,
                                 steps=200, n_s=25, seed=1),
    "c2_halos_2048": RunConfig("c2_halos_2048", n=2048, s=8, dt=5e-4,
                               steps=2000, n_s=50, seed=2),
    "c3_halos_sheet_8192": RunConfig("c3_halos_sheet_8192", n=8192, s=8,
                                     dt=2.5e-4, steps=4000, n_s=50, seed=3),
    # electron plasma on a ring (x periodic, G = -1/2, mean density 1):
    # two counter-streaming Maxwellian beams (v = +-2.4, unit dispersion)
    # with a 1 % density perturbation of wavenumber 0.2 -- the two-stream
    # instability, whose phase-space vortices wind the elements up
    "p2_two_stream_2048": RunConfig("p2_two_stream_2048", n=2048, s=8,
                                    dt=0.05, steps=2000, n_s=50, G=-0.5,
                                    box=(0.0, 10.0 * math.pi, -8.0, 8.0),
                                    seed=7, bc=1),
    "c5_halos_cold_16384": RunConfig("c5_halos_cold_16384", n=16384, s=16,
                                     dt=1.25e-4, steps=1000, n_s=20, seed=5),
}


def config(name: str, n: int | None = None) -> tuple[RunConfig, np.ndarray]:
    """Return (RunConfig, f0) for a named workload.  `n` optionally
    overrides the grid size (same recipe, same seed) for small test runs."""
    cfg = dataclasses.replace(CONFIGS[name])
    if n is not None:
        cfg.n = int(n)
    nx = nv = cfg.n
    box = cfg.box
    rng = np.random.default_rng(cfg.seed)
    if name.startswith("c1"):
        f = _unit_gaussian(nx, nv, box, 0.0, 0.0, 0.2, 0.2)
    elif name.startswith("c2"):
        f = halo_sum(nx, nv, box, rng, 4)
    elif name.startswith("c3"):
        k = int(rng.integers(3, 9))
        f = halo_sum(nx, nv, box, rng, k, mass=0.7)
        sheet = _sech2_sheet(nx, nv, box, 0.2, 0.1)
        # continuum mass of sech^2(x/0.2) exp(-v^2/0.02): 2*0.2 * sqrt(2 pi)*0.1
        f += 0.3 * sheet / (0.4 * math.sqrt(2.0 * math.pi) * 0.1)
    elif name.startswith("c5"):
        f = halo_sum(nx, nv, box, rng, 8, mass=0.8)
        f += 0.2 * _unit_gaussian(nx, nv, box, 0.0, 0.0, 0.2, 0.02)
    elif name.startswith("p2"):
        return cfg, two_stream(nx, nv, box, 0.2, 2.4, 0.01)
    else:
        raise KeyError(name)
    return cfg, finish(f, box, 1.0)


def landau4(ns: int, nv: int, L: float, vmax: float, alpha: float,
            seed: int = 0) -> np.ndarray:
    """4D phase space (x, y periodic on [0, L), u, w on [-vmax, vmax)): a
    Maxwellian plasma of mean density 1 with seeded perturbations of the
    four lowest Fourier modes (1, 0), (0, 1), (1, 1), (1, -1); array
    (w, u, y, x), the u and w edge rows zero."""
    rng = np.random.default_rng(seed)
    x = site_coords(ns, 0.0, L)
    u = site_coords(nv, -vmax, vmax)
    W_, U_, Y_, X_ = np.meshgrid(u, u, x, x, indexing="ij")
    pert = np.ones_like(X_)
    for mx, my in ((1, 0), (0, 1), (1, 1), (1, -1)):
        pert += alpha * rng.uniform(0.5, 1.0) * np.cos(
            2.0 * math.pi * (mx * X_ + my * Y_) / L + rng.uniform(0, 2 * math.pi))
    f = pert * np.exp(-0.5 * (U_ ** 2 + W_ ** 2)) / (2.0 * math.pi)
    f[0] = 0.0
    f[-1] = 0.0
    f[:, 0] = 0.0
    f[:, -1] = 0.0
    return f


def two_stream(nx: int, nv: int, box, k: float, v0: float,
               alpha: float) -> np.ndarray:
    """(1 + alpha cos(k x)) [N(v0, 1) + N(-v0, 1)] / 2 on a periodic box
    (no x edge ring: x wraps); the v edge rows are zeroed and the mean
    density over the box is 1."""
    x = site_coords(nx, box[0], box[1])
    v = site_coords(nv, box[2], box[3])
    X, V = np.meshgrid(x, v)
    beams = 0.5 * (np.exp(-0.5 * (V - v0) ** 2) + np.exp(-0.5 * (V + v0) ** 2))
    f = (1.0 + alpha * np.cos(k * X)) * beams / math.sqrt(2.0 * math.pi)
    f[0, :] = 0.0
    f[-1, :] = 0.0
    return f


def serving_requests(count: int = 512, base_seed: int = 4000,
                     sizes=(256, 512, 1024, 2048), strides=(4, 8),
                     steps=(200, 2000), remap=(25, 50)):
    """Independent runs for the serving loop: N uniform over `sizes`, stride
    over `strides`, steps ~ U{steps}, remap cadence ~ U{remap}, initial f a
    seeded sum of 1-6 Gaussian halos.  Returns a list of (RunConfig, f0)
    generators, one per request (f0 built lazily to bound host memory)."""
    out = []
    for r in range(count):
        rng = np.random.default_rng(base_seed + r)
        n = int(rng.choice(sizes))
        s = int(rng.choice(strides))
        nst = int(rng.integers(steps[0], steps[1] + 1))
        ns = int(rng.integers(remap[0], remap[1] + 1))
        k = int(rng.integers(1, 7))
        cfg = RunConfig(f"req{r}", n=n, s=s, dt=5e-4, steps=nst, n_s=ns,
                        seed=base_seed + r)
        out.append((cfg, k))
    return out


def request_f0(cfg: RunConfig, k: int) -> np.ndarray:
    """Initial f of one serving request (seeded by the request's own seed)."""
    rng = np.random.default_rng(cfg.seed + 1_000_000)
    return finish(halo_sum(cfg.n, cfg.n, cfg.box, rng, k), cfg.box, 1.0)
