"""Pins of the oracle's periodic variant (x periodic, force against a uniform
background; a plasma for G < 0, the gravitating "Jeans swindle" system for
G > 0): each against mathematics or physics that does not come from the
oracle.

* spline fit: the cyclic (1, 4, 1) system solved by FFT (circulant
  eigenvalues) along x and a dense solve along v; interpolation of the
  nodes; one period of shift changes nothing;
* six-point interpolation: equal to the plain interpolation of the data
  tiled three times;
* force: the sawtooth field of a point mass on a ring, zero for a uniform
  density, second-order convergence to the field of a cosine density;
* dynamics: free streaming wraps the elements exactly; the bucketed query
  equals brute force; linear Landau damping of a plasma (rate and frequency
  from the root of the kinetic dispersion relation) and the Jeans growth of
  a gravitating periodic system; total energy conserved; a translated
  initial condition gives the translated solution.
"""
import math

import numpy as np
import pytest

BOX = dict(x_min=0.0, v_min=-6.0, v_max=6.0)


def maxwell_ring(nx, nv, k, alpha):
    """f0 = (1 + alpha cos(k x)) exp(-v^2/2) / sqrt(2 pi) on one period."""
    L = 2.0 * math.pi / k
    x = (np.arange(nx) + 0.5) * L / nx
    v = -6.0 + (np.arange(nv) + 0.5) * 12.0 / nv
    X, V = np.meshgrid(x, v)
    f0 = (1.0 + alpha * np.cos(k * X)) * np.exp(-0.5 * V * V) / math.sqrt(
        2.0 * math.pi)
    return L, f0


def ring_params(nx, nv, L, s, G, dt, n_s, **kw):
    p = dict(nx=nx, nv=nv, x_max=L, sx=s, sv=s, G=G, dt=dt, n_s=n_s, bc=1,
             **BOX)
    p.update(kw)
    return p


# ------------------------------------------------------------- spline fit
def test_periodic_spline_equals_fft_and_dense_solve(orc):
    rng = np.random.default_rng(0)
    nx, nv = 24, 11
    F = rng.normal(size=(nv, nx))
    F[0, :] = F[-1, :] = 0.0
    C = orc.spline_fit(F, periodic=True)
    kk = np.arange(nx)
    lam = (4.0 + 2.0 * np.cos(2.0 * np.pi * kk / nx)) / 6.0
    T = np.real(np.fft.ifft(np.fft.fft(F, axis=1) / lam, axis=1))
    A = 4.0 * np.eye(nv) + np.eye(nv, k=1) + np.eye(nv, k=-1)
    A[0, 1] = 2.0
    A[-1, -2] = 2.0
    ref = np.linalg.solve(A, 6.0 * T)
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max()


def test_periodic_spline_interpolates_and_repeats(orc):
    rng = np.random.default_rng(1)
    nx, nv = 20, 9
    F = rng.normal(size=(nv, nx))
    F[0, :] = F[-1, :] = 0.0
    C = orc.spline_fit(F, periodic=True)
    for j in range(1, nv - 1):
        for i in range(nx):
            assert abs(orc.spline_eval(C, i, j, periodic=True) - F[j, i]) \
                <= 1e-13 * np.abs(F).max()
    # positions are clamped to [-12, nx + 11] sites; inside, one period of
    # shift changes nothing
    for _ in range(40):
        sx, sv = rng.uniform(-0.5, 11.0), rng.uniform(0.0, nv - 1.0)
        a = orc.spline_eval(C, sx, sv, periodic=True)
        b = orc.spline_eval(C, sx + nx, sv, periodic=True)
        assert abs(a - b) <= 1e-12 * np.abs(F).max()


def test_periodic_int1_equals_tiled_data(orc):
    rng = np.random.default_rng(2)
    nx, nv = 16, 10
    F = rng.normal(size=(nv, nx))
    tiled = np.concatenate([F, F, F], axis=1)
    for _ in range(200):
        sx = rng.uniform(-3.0, nx + 2.0)
        sv = rng.uniform(-1.0, nv)
        a = orc.int1(F, sx, sv, periodic=True)
        b = orc.int1(tiled, sx + nx, sv)
        assert abs(a - b) <= 1e-13 * (1.0 + abs(b))


# ------------------------------------------------------------------ force
def test_point_mass_sawtooth(orc):
    """da/dx = -2 G (rho - rho_bar) with zero mean: for one loaded cell the
    field is the periodic sawtooth, exact at the sites."""
    nx, L, G, M, m = 40, 3.0, 0.7, 2.5, 13
    o = orc.Oracle(**ring_params(nx, 16, L, 4, G, 0.01, 0))
    dx = L / nx
    rho = np.zeros(nx)
    rho[m] = M / dx
    a, da, d2a = o.poisson(rho)
    x = (np.arange(nx) + 0.5) * dx
    raw = G * M * (2.0 * x / L - 2.0 * (np.arange(nx) > m)
                   - 1.0 * (np.arange(nx) == m))
    ref = raw - raw.mean()
    assert np.abs(a - ref).max() <= 1e-13 * np.abs(ref).max()
    # the discrete slope between loaded cells is the background's, 2 G M / L
    assert np.allclose(da[m + 2:-1], 2.0 * G * M / L, rtol=1e-12)


def test_uniform_density_has_no_force(orc):
    o = orc.Oracle(**ring_params(32, 16, 2.0, 4, -0.5, 0.01, 0))
    a, da, d2a = o.poisson(np.full(32, 1.7))
    assert np.abs(a).max() <= 1e-13 and np.abs(da).max() <= 1e-11


def test_cosine_density_converges_at_second_order(orc):
    L, G, amp = 5.0, -0.5, 0.3
    errs = []
    for nx in (32, 64, 128):
        o = orc.Oracle(**ring_params(nx, 16, L, 4, G, 0.01, 0))
        x = (np.arange(nx) + 0.5) * L / nx
        kx = 2.0 * math.pi / L
        a, da, _ = o.poisson(1.0 + amp * np.cos(kx * x))
        exact = -2.0 * G * amp * np.sin(kx * x) / kx
        assert abs(a.sum()) <= 1e-12 * np.abs(exact).max() * nx
        errs.append(np.abs(a - exact).max())
        assert np.abs(da + 2.0 * G * amp * np.cos(kx * x)).max() <= 0.05
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 1.9), slopes


# --------------------------------------------------------------- dynamics
def test_free_streaming_wraps_elements(orc):
    nx, nv, s = 32, 32, 4
    L, f0 = maxwell_ring(nx, nv, 0.5, 0.1)
    p = ring_params(nx, nv, L, s, 0.0, 0.3, 0)
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    q = o.get_elements()
    o.step(40)
    t = o.t
    el = o.get_elements()
    want = np.mod(q[0] + q[1] * t, L)
    diff = np.abs(el[0] - want)
    diff = np.minimum(diff, L - diff)
    assert diff.max() <= 1e-12 * L
    assert np.all((el[0] >= 0.0) & (el[0] < L))
    assert np.abs(el[3] - t).max() <= 1e-13 * t
    assert np.array_equal(el[1], q[1])


def test_periodic_bucketed_query_equals_brute_force(orc):
    nx, nv, s = 48, 32, 4
    L, f0 = maxwell_ring(nx, nv, 2.0 * math.pi / 6.0, 0.2)
    o = orc.Oracle(**ring_params(nx, nv, L, s, -0.5, 0.05, 0))
    o.init_conditions(f0)
    o.step(6)
    rng = np.random.default_rng(4)
    el = o.get_elements()
    el[0] = np.mod(el[0] + rng.uniform(-0.2, 0.2, el.shape[1]) * L / nx, L)
    el[2:6] += rng.uniform(-0.05, 0.05, el[2:6].shape)
    o.set_elements(el)
    a = o.assignment(brute=False)
    b = o.assignment(brute=True)
    assert np.array_equal(a, b)
    # sites near both ends of the ring take elements from the other end
    x_el = el[0][a[:, 0][a[:, 0] >= 0]]
    assert np.any(x_el > 0.5 * L)


def _dispersion_root(k, G, guess):
    from scipy.optimize import fsolve
    from scipy.special import wofz

    def eps(w):
        z = w / (math.sqrt(2.0) * k)
        Z = 1j * math.sqrt(math.pi) * wofz(z)
        # rho_bar = 1, unit velocity dispersion
        return 1.0 - 2.0 * G / k ** 2 * (1.0 + z * Z)

    def f(xy):
        e = eps(xy[0] + 1j * xy[1])
        return [e.real, e.imag]

    wr, wi = fsolve(f, guess, xtol=1e-12)
    return wr, wi


@pytest.mark.slow
def test_landau_damping(orc):
    """Plasma (G = -1/2, mean density 1, a = -E): the k = 0.5 mode of a 1 %
    density perturbation damps at the rate and oscillates at the frequency
    of the root of 1 + (1 + zeta Z(zeta)) / k^2 = 0."""
    k = 0.5
    wr, wi = _dispersion_root(k, -0.5, [1.4, -0.15])
    L, f0 = maxwell_ring(64, 128, k, 0.01)
    o = orc.Oracle(**ring_params(64, 128, L, 4, -0.5, 0.1, 10))
    o.init_conditions(f0)
    e0 = o.diagnostics()["energy"]
    ts, W, E = [], [], []
    for _ in range(250):
        o.step(1)
        d = o.diagnostics()
        ts.append(d["t"])
        W.append(d["e_pot"])
        E.append(d["energy"])
    ts, W = np.array(ts), np.array(W)
    pk = [i for i in range(1, len(W) - 1) if W[i] > W[i - 1] and W[i] >= W[i + 1]]
    tp, wp = ts[pk], W[pk]
    sel = (tp > 1.0) & (tp < 22.0)
    gamma = np.polyfit(tp[sel], np.log(wp[sel]), 1)[0] / 2.0
    omega = math.pi / np.mean(np.diff(tp[sel]))
    assert abs(gamma - wi) <= 0.02 * abs(wi), (gamma, wi)
    assert abs(omega - wr) <= 0.01 * wr, (omega, wr)
    assert (max(E) - min(E)) <= 1e-5 * abs(e0)


@pytest.mark.slow
def test_jeans_growth(orc):
    """Gravitating ring (G > 0, the mean density removed): a mode longer than
    the Jeans length grows at the imaginary root of the same dispersion
    relation with the opposite sign of G."""
    k, G = 0.5, 0.25
    wr, wi = _dispersion_root(k, G, [0.0, 0.3])
    assert abs(wr) < 1e-8 and wi > 0.0
    L, f0 = maxwell_ring(64, 128, k, 1e-4)
    o = orc.Oracle(**ring_params(64, 128, L, 4, G, 0.05, 10))
    o.init_conditions(f0)
    ts, W = [], []
    for _ in range(120):
        o.step(1)
        d = o.diagnostics()
        ts.append(d["t"])
        W.append(-d["e_pot"])
    ts, W = np.array(ts), np.array(W)
    sel = (ts > 2.0) & (ts < 6.0)
    growth = np.polyfit(ts[sel], np.log(W[sel]), 1)[0] / 2.0
    assert abs(growth - wi) <= 0.02 * wi, (growth, wi)


def test_translated_initial_condition(orc):
    nx, nv, s = 32, 32, 4
    L, f0 = maxwell_ring(nx, nv, 2.0 * math.pi / 4.0, 0.3)
    p = ring_params(nx, nv, L, s, -0.5, 0.1, 5)
    a = orc.Oracle(**p)
    b = orc.Oracle(**p)
    shift = 2 * s
    a.init_conditions(f0)
    b.init_conditions(np.roll(f0, shift, axis=1))
    a.step(12)
    b.step(12)
    fa, fb = a.reconstruct_f(), b.reconstruct_f()
    assert np.abs(np.roll(fa, shift, axis=1) - fb).max() <= 1e-10 * np.abs(fa).max()
