"""Comparison rules of the GPU parity tests (engine through the C ABI
against the CPU oracle).

The FP64 engine evaluates every per-site and per-element formula with the
oracle's operations and roundings.  Two reductions are summed in different
orders: the column sums of the density projection (section 2.5) and the
cumulative mass of eq. (acccomp) are running sums from row / site 0 in the
oracle and blocked sums over the engine's tiles.  The force therefore
differs by rounding, and so do the elements it kicks.  The tests compare:

* f and rho: relative L-inf, max |diff| / max |oracle| <= RTOL = 1e-12;
* elements: the second-order maps P(Q) = P_m + T dQ + 1/2 dQ^T H dQ of the
  two element states over each element's validity window (|dQ_b| at most
  one element spacing per axis), in element spacings of the image axis
  (map_gap) <= MAP_TOL;
* the nearest-element assignment: bit for bit, given the same element
  state (assignment_same_state injects the oracle's elements into the
  engine first);
* the time and step size of a variable-step run: relative TIME_RTOL.

MAP_TOL: a difference of the column sums by a few ulps changes M_left, a
and a' at the ulp level, but the second difference a'' divides it by dx^2;
the H kick carries that into the map as 1/2 dt a'' dQ^2, about
dt G eps M_tot sqrt(nx) s^2 / (2 dv_m) element spacings per step (eps the
double-precision unit roundoff, s the element stride in sites), below
1e-12 for every tested workload (measured: 4e-15 after 70 steps of halos
at 512^2, 3e-13 after two steps of the 2048^2 plasma).  Elements are reset
at every resampling, so the difference accumulates over at most n_s steps;
MAP_TOL = 1e-10 element spacings covers the longest tested cycle.  A wrong
term anywhere in the element update moves the maps by many orders more.
"""
import numpy as np

RTOL = 1e-12
MAP_TOL = 1e-10
TIME_RTOL = 1e-12
EPS = 2.0 ** -53  # unit roundoff of double precision


def rel_linf(a, b):
    """max |a - b| / max |b| (max |a - b| when b is all zero)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    scale = np.abs(b).max() if b.size else 0.0
    d = np.abs(a - b).max() if b.size else 0.0
    return float(d / scale) if scale > 0 else float(d)


def force_close(got, ref, rho, o):
    """a, a', a'' of the engine against the oracle run o's for the same rho
    (lists of three arrays).  Both sides evaluate eq. (acccomp) and the
    finite differences with the same operations; only the cumulative masses
    are summed in different orders.  For n terms, two summation orders
    differ by at most 2 (n - 1) eps sum |terms|, so every M_left(i) by at
    most dM = 2 n eps dx sum |rho|.  a combines three cumulative masses (the
    periodic form B(i) - mean B, with the background term and the mean, at
    most ten dM), so |da| <= 12 |G| dM; a' and a'' take differences of two
    and four values of a over 2 dx and dx^2.  A few ulps of the largest
    |value| cover the final roundings."""
    n = o.nx
    dx = (o.p.get("x_max", 1.0) - o.p.get("x_min", -1.0)) / n
    G = abs(o.p.get("G", 1.0))
    dM = 2.0 * n * EPS * dx * float(np.abs(np.asarray(rho)).sum())
    ba = 12.0 * G * dM
    bounds = (ba, ba / dx, 4.0 * ba / (dx * dx))
    for name, x, y, b in zip(("a", "a'", "a''"), got, ref, bounds):
        x = np.asarray(x, np.float64)
        y = np.asarray(y, np.float64)
        tol = b + 4.0 * EPS * float(np.abs(y).max())
        d = float(np.abs(x - y).max())
        assert d <= tol, f"{name}: {d:.3e} > {tol:.3e}"


def map_gap(el_a, el_b, dxm, dvm):
    """Largest disagreement, in element spacings, of the second-order maps
    of two 2D element states (SoA [12][E]: x, v, Txx, Txv, Tvx, Tvv, Hx_xx,
    Hx_xv, Hx_vv, Hv_xx, Hv_xv, Hv_vv) over the validity windows
    |dq_x| <= dxm, |dq_v| <= dvm."""
    d = np.abs(np.asarray(el_a, np.float64) - np.asarray(el_b, np.float64))
    ex = (d[0] + d[2] * dxm + d[3] * dvm +
          0.5 * (d[6] * dxm * dxm + 2.0 * d[7] * dxm * dvm +
                 d[8] * dvm * dvm)) / dxm
    ev = (d[1] + d[4] * dxm + d[5] * dvm +
          0.5 * (d[9] * dxm * dxm + 2.0 * d[10] * dxm * dvm +
                 d[11] * dvm * dvm)) / dvm
    if ex.size == 0:
        return 0.0
    return float(max(ex.max(), ev.max()))


def spacings(o):
    """Element spacings (dx_m, dv_m) of a 2D oracle run."""
    p = o.p
    dxm = (p.get("x_max", 1.0) - p.get("x_min", -1.0)) / o.nx * o.sx
    dvm = (p.get("v_max", 1.0) - p.get("v_min", -1.0)) / o.nv * o.sv
    return dxm, dvm


def assert_elements_close(el_gpu, o, tol=MAP_TOL):
    """The engine's element state against the oracle run o's."""
    el_gpu = np.asarray(el_gpu)
    el_ref = o.get_elements()
    gap = map_gap(el_gpu, el_ref, *spacings(o))
    assert gap <= tol, f"element maps differ by {gap:.3e} element spacings"
    return gap


# 4D: H[a][bc] stored for b <= c in the order 00 01 02 03 11 12 13 22 23 33
_PAIRS4 = [(b, c) for b in range(4) for c in range(b, 4)]


def map_gap4(el_a, el_b, dm):
    """4D analogue of map_gap (SoA [60][E]: P (4), T row major (16), H
    (4 x 10)); dm = element spacings of the four axes."""
    d = np.abs(np.asarray(el_a, np.float64) - np.asarray(el_b, np.float64))
    worst = 0.0
    for a in range(4):
        e = d[a].copy()
        for b in range(4):
            e += d[4 + 4 * a + b] * dm[b]
        for k, (b, c) in enumerate(_PAIRS4):
            w = 1.0 if b == c else 2.0
            e += 0.5 * w * d[20 + 10 * a + k] * dm[b] * dm[c]
        if e.size:
            worst = max(worst, float((e / dm[a]).max()))
    return worst


def assignment_same_state(g, o, brute=False):
    """Inject the oracle's element state into the engine run g and return
    (engine assignment, oracle assignment) for that one state."""
    g.set_elements(o.get_elements())
    a_gpu = g.assignment().cpu().numpy()
    return a_gpu, o.assignment(brute)
