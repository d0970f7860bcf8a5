"""Pins of the 4D phase-space oracle (x, y periodic; u, w velocities) against
mathematics and physics that do not come from it:

* 15-point interpolation exact on quadratics in four variables, exact at
  the nodes, a partition of unity;
* inverse map exact for linear element maps, third-order error with a
  Hessian, A T = I;
* tensor spline fit equal to separable FFT (periodic axes) and dense
  (mirror axes) solves, interpolating the nodes;
* field of a cosine density equal to the spectral solution along x, along
  y and obliquely; no force for a uniform density;
* free streaming wraps the elements exactly and drifts injected T and H by
  t times their velocity rows; bucketed query = brute force; the validity
  window strict per axis, and the assignment of displaced undeformed
  elements (unmapped sites included) equal to a numpy brute force;
  exchanging x <-> y and u <-> w exchanges the solution; translation
  invariance; Landau damping at the kinetic rate with energy conserved.
"""
import math

import numpy as np
import pytest


@pytest.fixture(scope="module")
def v4(orc):
    import oracle.vp4 as v4
    return v4


def maxwell4(ns, nv, L, vmax, kx, ky, alpha):
    x = (np.arange(ns) + 0.5) * L / ns
    u = -vmax + (np.arange(nv) + 0.5) * 2.0 * vmax / nv
    W_, U_, Y_, X_ = np.meshgrid(u, u, x, x, indexing="ij")
    return (1.0 + alpha * np.cos(kx * X_ + ky * Y_)) * np.exp(
        -0.5 * (U_ ** 2 + W_ ** 2)) / (2.0 * math.pi)


def test_int15_exact_on_quadratics(v4):
    rng = np.random.default_rng(0)
    ns, nv = 10, 9
    idx = np.meshgrid(*[np.arange(n) for n in (nv, nv, ns, ns)], indexing="ij")
    l, k, j, i = [a.astype(float) for a in idx]
    for _ in range(5):
        c = rng.normal(size=15)
        v = [i, j, k, l]

        def q(p):
            s = c[0] + c[1] * p[0] + c[2] * p[1] + c[3] * p[2] + c[4] * p[3]
            n = 5
            for a in range(4):
                for b in range(a, 4):
                    s = s + c[n] * p[a] * p[b]
                    n += 1
            return s
        F = q(v)
        for _ in range(20):
            s4 = np.array([rng.uniform(2, ns - 3), rng.uniform(2, ns - 3),
                           rng.uniform(2, nv - 3), rng.uniform(2, nv - 3)])
            assert abs(v4.int15(F, s4) - q(s4)) <= 1e-11 * (1 + np.abs(F).max())


def test_int15_nodes_and_unity(v4):
    rng = np.random.default_rng(1)
    F = rng.normal(size=(6, 6, 8, 8))
    for _ in range(30):
        g = [int(rng.integers(0, 8)), int(rng.integers(0, 8)),
             int(rng.integers(0, 6)), int(rng.integers(0, 6))]
        assert v4.int15(F, np.array(g, float)) == F[g[3], g[2], g[1], g[0]]
    ones = np.ones((6, 6, 8, 8))
    for _ in range(30):
        s4 = np.array([rng.uniform(-3, 10), rng.uniform(-3, 10),
                       rng.uniform(1.5, 3.5), rng.uniform(1.5, 3.5)])
        assert abs(v4.int15(ones, s4) - 1.0) < 1e-14


def _element(rng, T, H, X):
    el = np.zeros(60)
    el[0:4] = X
    el[4:20] = T.ravel()
    el[20:60] = H.ravel()
    return el


def test_inverse_map_linear_exact_and_third_order(v4):
    rng = np.random.default_rng(2)
    Dm = np.full(4, 10.0)
    L = 1e6
    for _ in range(10):
        T = np.eye(4) + 0.3 * rng.normal(size=(4, 4))
        if np.linalg.det(T) <= 0:
            T[0] *= -1
        X = rng.normal(size=4)
        dQ = 0.1 * rng.normal(size=4)
        el = _element(rng, T, np.zeros((4, 10)), X)
        dq, valid, det = v4.inverse_map(el, Dm, X + T @ dQ, L)
        assert valid and abs(det - np.linalg.det(T)) <= 1e-12 * abs(det)
        assert np.abs(dq - dQ).max() <= 1e-13
    # with a Hessian: P = X + T dQ + 1/2 H(dQ, dQ); the map inverts to third
    # order in |dQ|
    T = np.eye(4) + 0.2 * rng.normal(size=(4, 4))
    H = 0.5 * rng.normal(size=(4, 10))
    X = rng.normal(size=4)
    pairs = [(b, c) for b in range(4) for c in range(b, 4)]
    d0 = rng.normal(size=4)
    d0 /= np.linalg.norm(d0)
    errs = []
    for h in (0.02, 0.01, 0.005):
        dQ = h * d0
        quad = np.array([sum(H[a, q] * dQ[b] * dQ[c] * (1 if b == c else 2)
                             for q, (b, c) in enumerate(pairs))
                         for a in range(4)])
        P = X + T @ dQ + 0.5 * quad
        dq, valid, _ = v4.inverse_map(_element(rng, T, H, X), Dm, P, L)
        errs.append(np.abs(dq - dQ).max())
    slopes = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(slopes > 2.7), slopes


def test_spline_fit_separable_solves(v4):
    rng = np.random.default_rng(3)
    ns, nv = 8, 6
    F = rng.normal(size=(nv, nv, ns, ns))
    F[0] = F[-1] = 0.0
    F[:, 0] = F[:, -1] = 0.0
    C = v4.spline_fit(F)
    lam = (4.0 + 2.0 * np.cos(2.0 * np.pi * np.arange(ns) / ns)) / 6.0
    ref = F.copy()
    for ax in (3, 2):  # x, y: circulant
        ref = np.real(np.fft.ifft(np.fft.fft(ref, axis=ax) /
                                  lam.reshape([-1 if a == ax else 1
                                               for a in range(4)]), axis=ax))
    M = 4.0 * np.eye(nv) + np.eye(nv, k=1) + np.eye(nv, k=-1)
    M[0, 1] = 2.0
    M[-1, -2] = 2.0
    Minv6 = 6.0 * np.linalg.inv(M)
    ref = np.einsum("kK,lKji->lkji", Minv6, ref)
    ref = np.einsum("lL,Lkji->lkji", Minv6, ref)
    assert np.abs(C - ref).max() <= 1e-12 * np.abs(ref).max()
    for _ in range(30):
        g = [int(rng.integers(0, ns)), int(rng.integers(0, ns)),
             int(rng.integers(1, nv - 1)), int(rng.integers(1, nv - 1))]
        got = v4.spline_eval(C, np.array(g, float))
        assert abs(got - F[g[3], g[2], g[1], g[0]]) <= 1e-12 * np.abs(F).max()


@pytest.mark.parametrize("mx,my", [(1, 0), (0, 1), (1, 1), (2, 1)])
def test_field_spectral_exact(v4, mx, my):
    ns, L, G, amp = 16, 5.0, -0.5, 0.3
    o = v4.Oracle4(ns=ns, nv=4, L=L, vmax=1.0, ss=4, sv=4, G=G, dt=0.1)
    x = (np.arange(ns) + 0.5) * L / ns
    Y, X = np.meshgrid(x, x, indexing="ij")
    kx, ky = 2 * np.pi * mx / L, 2 * np.pi * my / L
    ph = kx * X + ky * Y
    ax, ay = o.field(1.0 + amp * np.cos(ph))
    # phi = -2 G amp cos / |k|^2, a = -grad phi
    k2 = kx * kx + ky * ky
    ex = -2.0 * G * amp * kx * np.sin(ph) / k2
    ey = -2.0 * G * amp * ky * np.sin(ph) / k2
    assert np.abs(ax - ex).max() <= 1e-12 and np.abs(ay - ey).max() <= 1e-12
    ax0, ay0 = o.field(np.full((ns, ns), 1.7))
    assert np.abs(ax0).max() <= 1e-13 and np.abs(ay0).max() <= 1e-13


def test_free_streaming_wraps(v4):
    ns, nv, L, vmax = 16, 8, 4.0, 3.0
    o = v4.Oracle4(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=0.0, dt=0.3)
    o.init_conditions(maxwell4(ns, nv, L, vmax, 2 * np.pi / L, 0.0, 0.1))
    q = o.get_elements()
    o.step(10)
    t = o.t
    el = o.get_elements()
    for a in range(2):
        want = np.mod(q[a] + q[a + 2] * t, L)
        d = np.abs(el[a] - want)
        assert np.minimum(d, L - d).max() <= 1e-12 * L
    # T_x,u = T_y,w = t
    assert np.abs(el[4 + 2] - t).max() <= 1e-13 * t
    assert np.abs(el[4 + 4 + 3] - t).max() <= 1e-13 * t


def test_bucketed_equals_brute(v4):
    ns, nv, L, vmax = 16, 8, 4.0, 3.0
    o = v4.Oracle4(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=-0.5, dt=0.2)
    o.init_conditions(maxwell4(ns, nv, L, vmax, 2 * np.pi / L, 0.0, 0.2))
    o.step(3)
    rng = np.random.default_rng(4)
    el = o.get_elements()
    el[4:20] += rng.uniform(-0.05, 0.05, el[4:20].shape)
    el[0:2] = np.mod(el[0:2] + rng.uniform(-0.05, 0.05, el[0:2].shape), L)
    o.set_elements(el)
    assert np.array_equal(o.assignment(False), o.assignment(True))


def test_xy_exchange_symmetry(v4):
    """A mode along y evolves as the transposed mode along x."""
    ns, nv, L, vmax = 16, 8, 4.0 * math.pi, 6.0
    p = dict(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=-0.5, dt=0.2, n_s=3)
    a, b = v4.Oracle4(**p), v4.Oracle4(**p)
    fa = maxwell4(ns, nv, L, vmax, 0.5, 0.0, 0.05)
    a.init_conditions(fa)
    b.init_conditions(np.transpose(fa, (1, 0, 3, 2)))
    a.step(5)
    b.step(5)
    ga = a.reconstruct_f()
    gb = np.transpose(b.reconstruct_f(), (1, 0, 3, 2))
    assert np.abs(ga - gb).max() <= 1e-10 * np.abs(ga).max()


def test_translation_invariance(v4):
    ns, nv, L, vmax = 16, 8, 4.0 * math.pi, 6.0
    p = dict(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=-0.5, dt=0.2, n_s=3)
    a, b = v4.Oracle4(**p), v4.Oracle4(**p)
    f0 = maxwell4(ns, nv, L, vmax, 0.5, 0.5, 0.05)
    a.init_conditions(f0)
    b.init_conditions(np.roll(np.roll(f0, 4, axis=3), 8, axis=2))
    a.step(5)
    b.step(5)
    ga = np.roll(np.roll(a.reconstruct_f(), 4, axis=3), 8, axis=2)
    assert np.abs(ga - b.reconstruct_f()).max() <= 1e-10 * np.abs(ga).max()


@pytest.mark.slow
def test_landau_damping_4d(v4):
    """Plasma in 2D space (G = -1/2, mean density 1): a k = 0.5 density
    mode of a Maxwellian damps at the kinetic rate (the root of
    1 + (1 + zeta Z(zeta)) / k^2 = 0, -0.1534) within 5 % on a 16^4 grid,
    with the total energy conserved."""
    from scipy.optimize import fsolve
    from scipy.special import wofz
    k = 0.5

    def f(xy):
        z = (xy[0] + 1j * xy[1]) / (math.sqrt(2.0) * k)
        e = 1.0 + (1.0 + z * 1j * math.sqrt(math.pi) * wofz(z)) / k ** 2
        return [e.real, e.imag]
    wr, wi = fsolve(f, [1.4, -0.15], xtol=1e-12)
    ns, nv, L, vmax = 16, 16, 4.0 * math.pi, 6.0
    o = v4.Oracle4(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=-0.5, dt=0.2,
                   n_s=5)
    o.init_conditions(maxwell4(ns, nv, L, vmax, k, 0.0, 0.01))
    e0 = o.diagnostics()["energy"]
    ts, W, E = [], [], []
    for _ in range(60):
        o.step(1)
        d = o.diagnostics()
        ts.append(d["t"])
        W.append(d["e_pot"])
        E.append(d["energy"])
    ts, W = np.array(ts), np.array(W)
    pk = [i for i in range(1, len(W) - 1) if W[i] > W[i - 1] and W[i] >= W[i + 1]]
    tp, wp = ts[pk], W[pk]
    gamma = np.polyfit(tp, np.log(wp), 1)[0] / 2.0
    assert abs(gamma - wi) <= 0.05 * abs(wi), (gamma, wi)
    assert (max(E) - min(E)) <= 1e-4 * abs(e0)


def test_free_streaming_drifts_T_and_H(v4):
    """G = 0: only the drifts act, and they move the space rows of T and H
    by t times the velocity rows (the drift of the derivatives, section 2.4
    per component), on injected random T and H."""
    ns, nv, L, vmax, dt, n = 16, 8, 4.0, 3.0, 0.25, 8
    o = v4.Oracle4(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=0.0, dt=dt,
                   n_s=0)
    o.init_conditions(maxwell4(ns, nv, L, vmax, 2 * np.pi / L, 0.0, 0.1))
    rng = np.random.default_rng(9)
    el = o.get_elements()
    E = el.shape[1]
    el[4:20] += rng.uniform(-0.05, 0.05, (16, E))
    el[20:60] = rng.uniform(-0.2, 0.2, (40, E))
    o.set_elements(el)
    o.step(n)
    t = n * dt
    got = o.get_elements()
    for a in range(2):
        for b in range(4):
            want = el[4 + 4 * a + b] + t * el[4 + 4 * (a + 2) + b]
            assert np.abs(got[4 + 4 * a + b] - want).max() <= 1e-13
            assert np.array_equal(got[4 + 4 * (a + 2) + b],
                                  el[4 + 4 * (a + 2) + b])
        for q in range(10):
            want = el[20 + 10 * a + q] + t * el[20 + 10 * (a + 2) + q]
            assert np.abs(got[20 + 10 * a + q] - want).max() <= 1e-13
            assert np.array_equal(got[20 + 10 * (a + 2) + q],
                                  el[20 + 10 * (a + 2) + q])


def test_validity_window_and_unmapped_sites(v4):
    """The window |A (P - P_m)| < spacing is strict and per axis: an
    element is valid inside, not on the edge, not beyond.  With T = I and
    H = 0 injected and every element moved, the nearest valid element of
    every site (smallest (d^2, id), x and y periodic, -1 when none) equals a
    numpy brute force over that definition."""
    Dm = np.array([2.0, 2.0, 1.0, 1.0])
    X = np.array([1.0, -1.0, 0.5, 0.25])
    el = np.zeros(60)
    el[0:4] = X
    el[4:20] = np.eye(4).ravel()
    for off, want in ((0.99, True), (1.0, False), (1.01, False)):
        for a in range(4):
            P = X.copy()
            P[a] += off * Dm[a]
            assert v4.inverse_map(el, Dm, P, 1e6)[1] == want, (a, off)
    ns, nv, L, vmax = 16, 8, 4.0, 2.0
    o = v4.Oracle4(ns=ns, nv=nv, L=L, vmax=vmax, ss=4, sv=4, G=0.0, dt=0.1)
    o.init_conditions(maxwell4(ns, nv, L, vmax, 2 * np.pi / L, 0.0, 0.1))
    rng = np.random.default_rng(12)
    els = o.get_elements()
    E = els.shape[1]
    dxs, dus = L / ns, 2 * vmax / nv
    sp = np.array([4 * dxs, 4 * dxs, 4 * dus, 4 * dus])
    els[0:2] = np.mod(els[0:2] + rng.uniform(-0.7, 0.7, (2, E)) * sp[:2, None], L)
    els[2:4] += rng.uniform(-0.7, 0.7, (2, E)) * sp[2:, None]
    els[2] += 1.5 * sp[2]  # the lowest u rows lose every window
    els[4:20] = np.eye(4).ravel()[:, None]
    els[20:60] = 0.0
    o.set_elements(els)
    got = o.assignment(True)
    x = (np.arange(ns) + 0.5) * dxs
    u = -vmax + (np.arange(nv) + 0.5) * dus
    W_, U_, Y_, X_ = np.meshgrid(u, u, x, x, indexing="ij")
    P = np.stack([X_, Y_, U_, W_], -1)                     # (nv, nv, ns, ns, 4)
    d = P[..., None, :] - els[0:4].T                       # (..., E, 4)
    d[..., :2] -= L * np.round(d[..., :2] / L)
    valid = np.all(np.abs(d) < sp, axis=-1)
    d2 = np.where(valid, np.sum((d / sp) ** 2, axis=-1), np.inf)
    want = np.where(np.isfinite(d2.min(-1)), np.argmin(d2, axis=-1), -1)
    assert (want == -1).any() and (want >= 0).any()
    assert np.array_equal(got, want)
