"""Pins of the CPU oracle against what the paper and the mathematics fix.

Each test checks the oracle against something other than itself: closed
forms, exact reproduction properties, library routines, brute force, and the
few numbers the paper prints.  A plausible slip in the oracle (a dropped term,
a sign, an index, a transposed operand) fails at least one of them.
"""
import json
import math
import os

import numpy as np
import pytest

import workloads as W

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def box_params(n, s, dt=1e-3, n_s=0, G=1.0, nv=None, sv=None, **kw):
    p = dict(nx=n, nv=nv or n, x_min=-1.0, x_max=1.0, v_min=-1.0, v_max=1.0,
             sx=s, sv=sv or s, G=G, dt=dt, n_s=n_s)
    p.update(kw)
    return p


# ----------------------------------------------------------- interpolation
def test_int1_reproduces_quadratics(orc):
    """The six-point interpolation (section 2.2.1) is exact on quadratics;
    it pins the sign of the F(i_n - 1) terms and the v-row index."""
    rng = np.random.default_rng(0)
    nx, nv = 17, 13
    I, J = np.meshgrid(np.arange(nx), np.arange(nv))
    for _ in range(20):
        c = rng.normal(size=6)
        q = lambda x, v: (c[0] + c[1] * x + c[2] * v + c[3] * x * x
                          + c[4] * x * v + c[5] * v * v)
        F = q(I.astype(float), J.astype(float))
        for _ in range(30):
            sx = rng.uniform(2.0, nx - 3.0)
            sv = rng.uniform(2.0, nv - 3.0)
            got = orc.int1(F, sx, sv)
            assert abs(got - q(sx, sv)) <= 1e-12 * (1 + abs(F).max())


def test_int1_nodes_and_partition_of_unity(orc):
    rng = np.random.default_rng(1)
    F = rng.normal(size=(9, 11))
    for j in range(9):
        for i in range(11):
            assert orc.int1(F, float(i), float(j)) == F[j, i]
    ones = np.ones((9, 11))
    for _ in range(50):
        sx, sv = rng.uniform(1.5, 8.5), rng.uniform(1.5, 6.5)
        assert abs(orc.int1(ones, sx, sv) - 1.0) < 1e-15
    # outside the grid the data are zero
    assert orc.int1(ones, -2.6, 4.0) == 0.0
    assert orc.int1(ones, 4.0, 9.0 + 1.6) == 0.0


def test_monaghan_kernel(orc):
    """W of section 2.3.2: W(0)=1, W(1)=1/4, W(2)=0, compact support, and C2
    continuity at the joints x = 1 and x = 2."""
    assert orc.W(0.0) == 1.0
    assert orc.W(1.0) == 0.25
    assert orc.W(2.0) == 0.0
    assert orc.W(2.5) == 0.0
    h = 1e-4
    for x0 in (1.0, 2.0):
        left = [orc.W(x0 - k * h) for k in range(3)]
        right = [orc.W(x0 + k * h) for k in range(3)]
        d1l = (left[0] - left[1]) / h
        d1r = (right[1] - right[0]) / h
        assert abs(d1l - d1r) < 1e-3
        d2l = (left[0] - 2 * left[1] + left[2]) / h ** 2
        d2r = (right[2] - 2 * right[1] + right[0]) / h ** 2
        assert abs(d2l - d2r) < 1e-2
    # monotone decreasing on [0, 2]
    xs = np.linspace(0, 2, 201)
    ws = np.array([orc.W(x) for x in xs])
    assert np.all(np.diff(ws) <= 1e-15)


# ------------------------------------------------------------------ spline
def _forward_spline_nodes(c):
    """Node values of a cubic B-spline with coefficients c and mirror ghosts
    c(-1) = c(1), c(n) = c(n-2), along both axes: (c[i-1]+4c[i]+c[i+1])/6."""
    def along(a, axis):
        a = np.moveaxis(a, axis, 0)
        g = np.concatenate([a[1:2], a, a[-2:-1]], axis=0)
        out = (g[:-2] + 4 * g[1:-1] + g[2:]) / 6.0
        return np.moveaxis(out, 0, axis)
    return along(along(c, 1), 0)


def test_spline_fit_recovers_coefficients(orc):
    rng = np.random.default_rng(2)
    c = rng.normal(size=(12, 15))
    F = _forward_spline_nodes(c)
    got = orc.spline_fit(F)
    assert np.max(np.abs(got - c)) < 1e-13


def test_spline_fit_matches_dense_solve(orc):
    rng = np.random.default_rng(3)
    F = rng.normal(size=(10, 14))

    def mat(n):
        A = np.diag(np.full(n, 4.0)) + np.diag(np.ones(n - 1), 1) + \
            np.diag(np.ones(n - 1), -1)
        A[0, 1] = 2.0
        A[-1, -2] = 2.0
        return A
    T = np.linalg.solve(mat(14), 6.0 * F.T).T          # along x per row
    Cd = np.linalg.solve(mat(10), 6.0 * T)             # along v per column
    got = orc.spline_fit(F)
    assert np.max(np.abs(got - Cd)) < 1e-13


def test_spline_interpolates_nodes_and_converges_fourth_order(orc):
    rng = np.random.default_rng(4)
    F = rng.normal(size=(11, 13))
    F[0, :] = F[-1, :] = F[:, 0] = F[:, -1] = 0.0
    Cc = orc.spline_fit(F)
    for j in range(11):
        for i in range(13):
            assert abs(orc.spline_eval(Cc, i, j) - F[j, i]) < 1e-13
    # outside [0, n-1] the spline is zero
    assert orc.spline_eval(Cc, -0.01, 3.0) == 0.0
    assert orc.spline_eval(Cc, 3.0, 10.01) == 0.0

    # g vanishes with zero slope at both end nodes, like the edge
    # conditions of section 2.2.2; the error must fall like h^4.
    def err(n):
        t = np.arange(n) / (n - 1.0)
        g1 = np.sin(np.pi * t) ** 2
        G2 = np.outer(g1, g1)
        Cn = orc.spline_fit(G2)
        pts = np.random.default_rng(5).uniform(0, n - 1, size=(200, 2))
        e = 0.0
        for sx, sv in pts:
            exact = (np.sin(np.pi * sx / (n - 1)) ** 2
                     * np.sin(np.pi * sv / (n - 1)) ** 2)
            e = max(e, abs(orc.spline_eval(Cn, sx, sv) - exact))
        return e
    e1, e2 = err(24), err(48)
    assert e1 / e2 > 2 ** 3.5


def test_spline_mirror_symmetry(orc):
    rng = np.random.default_rng(6)
    F = rng.normal(size=(9, 12))
    F = F + F[:, ::-1]
    Cc = orc.spline_fit(F)
    assert np.max(np.abs(Cc - Cc[:, ::-1])) < 1e-13


# ---------------------------------------------------------- inverse map
def _random_T(rng, scale=0.6):
    th = rng.uniform(0, 2 * np.pi)
    R = np.array([[np.cos(th), -np.sin(th)], [np.sin(th), np.cos(th)]])
    a = np.exp(rng.uniform(-scale, scale))
    S = np.array([[1.0, rng.uniform(-scale, scale)], [0.0, 1.0]])
    return R @ np.diag([a, 1 / a]) @ S


def test_inverse_map_round_trip_third_order(orc):
    """Forward second-order map (section 2.1) followed by the oracle's
    inverse map (eq. QofP) leaves an O(|dQ|^3) residual."""
    rng = np.random.default_rng(7)
    for _ in range(10):
        T = _random_T(rng)
        H = rng.normal(size=6)          # Hx[xx,xv,vv], Hv[xx,xv,vv]
        Pm = rng.normal(size=2) * 0.1
        el = np.concatenate([Pm, T.ravel(), H])
        d = rng.normal(size=2)
        d /= np.linalg.norm(d)
        errs = []
        epss = [1e-2, 5e-3, 2.5e-3]
        for eps in epss:
            dq = eps * d
            quad = lambda h: (h[0] * dq[0] ** 2 + 2 * h[1] * dq[0] * dq[1]
                              + h[2] * dq[1] ** 2)
            P = Pm + T @ dq + 0.5 * np.array([quad(H[:3]), quad(H[3:])])
            gx, gv, valid, det = orc.inverse_map(el, 1.0, 1.0, P[0], P[1])
            assert abs(det - 1.0) < 1e-12
            errs.append(np.hypot(gx - dq[0], gv - dq[1]))
        slope = np.log(errs[0] / errs[2]) / np.log(epss[0] / epss[2])
        assert 2.7 < slope < 3.3, (errs, slope)


def test_inverse_map_linear_exact_and_validity(orc):
    rng = np.random.default_rng(8)
    T = _random_T(rng)
    el = np.concatenate([[0.1, -0.2], T.ravel(), np.zeros(6)])
    dq = np.array([0.3, -0.2])
    P = el[:2] + T @ dq
    gx, gv, valid, _ = orc.inverse_map(el, 1.0, 1.0, P[0], P[1])
    assert abs(gx - dq[0]) < 1e-14 and abs(gv - dq[1]) < 1e-14 and valid
    # validity is strict: |l| < spacing
    P = el[:2] + T @ np.array([1.5, 0.0])
    assert not orc.inverse_map(el, 1.0, 1.0, P[0], P[1])[2]


# ------------------------------------------------------------ the query
def _perturbed_state(o, rng, amp_x=0.3, amp_t=0.15, amp_h=2.0):
    el = o.get_elements()
    E = el.shape[1]
    dxm = 2.0 / o.nx * o.sx
    el[0] += rng.uniform(-amp_x, amp_x, E) * dxm
    el[1] += rng.uniform(-amp_x, amp_x, E) * dxm
    el[2] += rng.uniform(-amp_t, amp_t, E)
    el[3] += rng.uniform(-amp_t, amp_t, E)
    el[4] += rng.uniform(-amp_t, amp_t, E)
    el[5] += rng.uniform(-amp_t, amp_t, E)
    el[6:] = rng.uniform(-amp_h, amp_h, (6, E))
    return el


@pytest.mark.parametrize("n,s,nv,sv", [(16, 4, 16, 4), (32, 4, 24, 2),
                                       (48, 8, 64, 8), (40, 2, 32, 4)])
def test_bucketed_query_equals_brute_force(orc, n, s, nv, sv):
    rng = np.random.default_rng(n * 100 + s)
    o = orc.Oracle(**box_params(n, s, nv=nv, sv=sv))
    o.init_conditions(np.ones((nv, n)))
    for trial in range(3):
        el = _perturbed_state(o, rng) if trial else o.get_elements()
        o.set_elements(el)
        a_b = o.assignment(brute=True)
        a_q = o.assignment(brute=False)
        assert np.array_equal(a_b, a_q)
        if trial == 0:
            assert (a_b >= 0).all()


def test_query_exact_ties_go_to_lowest_id(orc):
    """At t = 0 a site midway between elements is an exact binary tie; the
    nearest element is the one with the lowest id."""
    n, s = 32, 4
    o = orc.Oracle(**box_params(n, s))
    o.init_conditions(np.ones((n, n)))
    a = o.assignment(brute=False)
    M = n // s
    # element k sits on site s*k + s/2; site s*k + s/2 + s/2 is midway
    # between k and k+1 (x tie) -> k; same along v -> row l.
    for l in range(M - 1):
        for k in range(M - 1):
            i = s * k + s // 2
            j = s * l + s // 2
            assert a[j, i] == l * M + k                    # on the element
            assert a[j, i + s // 2] == l * M + k           # x tie
            assert a[j + s // 2, i] == l * M + k           # v tie
            assert a[j + s // 2, i + s // 2] == l * M + k  # 4-way tie
            assert a[j, i + s // 2 + 1] == l * M + k + 1   # just past it


# ------------------------------------------------------------ the field
def test_poisson_point_mass(orc):
    n = 64
    o = orc.Oracle(**box_params(n, 4, G=1.5))
    dx = 2.0 / n
    rho = np.zeros(n)
    i0, m0 = 20, 0.7
    rho[i0] = m0 / dx
    a, da, d2a = o.poisson(rho)
    GM = 1.5 * m0
    assert np.allclose(a[:i0], GM, rtol=0, atol=1e-14)
    assert abs(a[i0]) < 1e-14
    assert np.allclose(a[i0 + 1:], -GM, rtol=0, atol=1e-14)


def test_poisson_antisymmetry_and_slab_gradient(orc):
    """a = G (M_right - M_left) of eq. (acccomp): antisymmetric for a
    symmetric density, and da/dx = -2 G rho0 inside a uniform slab, which
    pins the centred difference over 2 dx (reading R12)."""
    n = 128
    G = 0.8
    o = orc.Oracle(**box_params(n, 4, G=G))
    x = W.site_coords(n, -1, 1)
    rho = np.exp(-x ** 2 / 0.1)
    a, da, d2a = o.poisson(rho)
    assert np.max(np.abs(a + a[::-1])) < 1e-14
    rho0 = 0.37
    rho = np.where(np.abs(x) < 0.5, rho0, 0.0)
    a, da, d2a = o.poisson(rho)
    inner = np.abs(x) < 0.45
    assert np.allclose(da[inner], -2 * G * rho0, rtol=1e-12, atol=0)
    assert np.max(np.abs(d2a[inner])) < 1e-8
    # total: a -> +G M left of the mass, -G M right of it
    M = rho.sum() * (2.0 / n)
    assert abs(a[0] - G * M) < 1e-14 and abs(a[-1] + G * M) < 1e-14


def test_tsc_reproduces_linear_fields(orc):
    """Dual TSC weights of section 2.5 sum to one and reproduce a linear
    field exactly."""
    g = 0.3 + 0.7 * np.arange(20.0)
    for u in np.linspace(2.0, 17.0, 41):
        assert abs(orc.tsc(g, u) - (0.3 + 0.7 * u)) < 1e-12
    assert abs(orc.tsc(np.ones(20), 7.3) - 1.0) < 1e-15


# ------------------------------------------------------ element motion
def test_free_streaming_elements_closed_form(orc):
    """G = 0: x = q_x + q_v t, T = [[1, t], [0, 1]], H = 0 (section 2.4)."""
    n, s, dt, k = 32, 4, 0.01, 7
    o = orc.Oracle(**box_params(n, s, dt=dt, G=0.0))
    o.init_conditions(np.zeros((n, n)))
    q = o.get_elements()
    o.step(k)
    el = o.get_elements()
    t = k * dt
    assert np.allclose(el[0], q[0] + q[1] * t, rtol=0, atol=1e-15)
    assert np.array_equal(el[1], q[1])
    assert np.allclose(el[3], t, rtol=0, atol=1e-15)
    assert np.array_equal(el[2], np.ones_like(el[2]))
    assert np.array_equal(el[4], np.zeros_like(el[4]))
    assert np.array_equal(el[5], np.ones_like(el[5]))
    assert not el[6:].any()


def test_constant_force_leapfrog_exact(orc):
    """Drift-kick-drift is exact for a constant force a0."""
    n, s, dt, k, a0 = 32, 4, 0.01, 9, -0.35
    o = orc.Oracle(**box_params(n, s, dt=dt, force_mode=orc.FORCE_EXTERNAL,
                                ext=(a0, 0.0, 0.0)))
    o.init_conditions(np.zeros((n, n)))
    q = o.get_elements()
    o.step(k)
    el = o.get_elements()
    t = k * dt
    assert np.allclose(el[0], q[0] + q[1] * t + 0.5 * a0 * t * t, rtol=0,
                       atol=1e-14)
    assert np.allclose(el[1], q[1] + a0 * t, rtol=0, atol=1e-14)
    assert np.allclose(el[3], t, rtol=0, atol=1e-15)
    assert not el[4].any() and not el[6:].any()


def test_harmonic_force_deformation_tensor(orc):
    """a = -w^2 x: T after k steps equals the k-th power of the one-step
    drift-kick-drift matrix; this pins the T kick (reading R5), whose
    printed right-hand side uses the wrong component."""
    n, s, dt, k, w2 = 32, 4, 0.02, 25, 3.0
    o = orc.Oracle(**box_params(n, s, dt=dt, force_mode=orc.FORCE_EXTERNAL,
                                ext=(0.0, -w2, 0.0)))
    o.init_conditions(np.zeros((n, n)))
    o.step(k)
    el = o.get_elements()
    h = 0.5 * dt
    D = np.array([[1.0, h], [0.0, 1.0]])
    K = np.array([[1.0, 0.0], [-w2 * dt, 1.0]])
    Mk = np.linalg.matrix_power(D @ K @ D, k)
    for comp, val in zip((2, 3, 4, 5), Mk.ravel()):
        assert np.allclose(el[comp], val, rtol=0, atol=1e-13)
    det = el[2] * el[5] - el[3] * el[4]
    assert np.max(np.abs(det - 1)) < 1e-13
    assert not el[6:].any()


def _dkd_particle(q, dt, k, acc):
    """Drift-kick-drift map of one particle (x, v) under the force acc(x)."""
    x, v = q
    for _ in range(k):
        x = x + 0.5 * dt * v
        v = v + dt * acc(x)
        x = x + 0.5 * dt * v
    return np.array([x, v])


def test_T_and_H_are_derivatives_of_the_discrete_map(orc):
    """With an analytic force a = a0 + a1 x + a2 x^2 the element's T and H
    after k steps are the exact Jacobian and Hessian of the discrete
    drift-kick-drift map of its particle (section 2.4 equations of motion,
    discretised as in the predictor/kick/corrector).  Checked against
    central finite differences of the particle map."""
    n, s, dt, k = 32, 8, 0.02, 15
    a0, a1, a2 = 0.1, -1.3, 2.1
    o = orc.Oracle(**box_params(n, s, dt=dt, force_mode=orc.FORCE_EXTERNAL,
                                ext=(a0, a1, a2)))
    o.init_conditions(np.zeros((n, n)))
    q0 = o.get_elements()[:2].copy()
    o.step(k)
    el = o.get_elements()
    acc = lambda x: a0 + a1 * x + a2 * x * x
    eps = 1e-4
    for e in (0, 5, 11, q0.shape[1] - 1):
        Q = q0[:, e]
        P = lambda dq: _dkd_particle(Q + dq, dt, k, acc)
        assert np.allclose(P(np.zeros(2)), el[:2, e], rtol=0, atol=1e-13)
        ex, ev = np.array([eps, 0.0]), np.array([0.0, eps])
        Tx = (P(ex) - P(-ex)) / (2 * eps)
        Tv = (P(ev) - P(-ev)) / (2 * eps)
        Hxx = (P(ex) - 2 * P(np.zeros(2)) + P(-ex)) / eps ** 2
        Hvv = (P(ev) - 2 * P(np.zeros(2)) + P(-ev)) / eps ** 2
        Hxv = (P(ex + ev) - P(ex - ev) - P(-ex + ev) + P(-ex - ev)) / (4 * eps ** 2)
        T = np.array([[Tx[0], Tv[0]], [Tx[1], Tv[1]]])
        assert np.allclose(el[2:6, e], T.ravel(), rtol=0, atol=1e-7)
        H = np.array([Hxx[0], Hxv[0], Hvv[0], Hxx[1], Hxv[1], Hvv[1]])
        assert np.allclose(el[6:12, e], H, rtol=0, atol=1e-5 * (1 + abs(H).max()))
        assert np.abs(H).max() > 1e-2


def test_harmonic_well_reconstruction_closed_form(orc):
    """a = -w^2 x: the discrete flow is linear, P = M^k Q, so the exact
    transported density is f0(M^-k P); the reconstruction must follow it
    within the second-order interpolation error (exercises every entry of
    A = T^-1 with T_xx != T_vv)."""
    n, s, dt, k, w2 = 128, 4, 0.02, 20, 2.0
    o = orc.Oracle(**box_params(n, s, dt=dt, n_s=0,
                                force_mode=orc.FORCE_EXTERNAL,
                                ext=(0.0, -w2, 0.0)))
    box = (-1, 1, -1, 1)
    sig = 0.15
    f0 = W.finish(W.gaussian_blob(n, n, box, 0.1, -0.05, sig, sig), box,
                  mass=None)
    o.init_conditions(f0)
    o.step(k)
    f = o.reconstruct_f()
    h = 0.5 * dt
    D = np.array([[1.0, h], [0.0, 1.0]])
    K = np.array([[1.0, 0.0], [-w2 * dt, 1.0]])
    Minv = np.linalg.inv(np.linalg.matrix_power(D @ K @ D, k))
    x = W.site_coords(n, -1, 1)[None, :]
    v = W.site_coords(n, -1, 1)[:, None]
    qx = Minv[0, 0] * x + Minv[0, 1] * v
    qv = Minv[1, 0] * x + Minv[1, 1] * v
    exact = np.exp(-0.5 * ((qx - 0.1) / sig) ** 2 - 0.5 * ((qv + 0.05) / sig) ** 2)
    assert np.abs(f - exact).max() < 5e-3


def test_anharmonic_reconstruction_follows_reversed_map(orc):
    """a = a0 + a1 x + a2 x^2: the discrete map is undone exactly by running
    the same leapfrog with -dt, so f(P) must equal f0 at the reversed
    position within the interpolation and second-order map errors.  Here
    T_xx != T_vv and every entry of A = T^-1 matters."""
    n, s, dt, k = 128, 4, 0.02, 15
    a0, a1, a2 = 0.1, -1.3, 2.1
    o = orc.Oracle(**box_params(n, s, dt=dt, n_s=0,
                                force_mode=orc.FORCE_EXTERNAL,
                                ext=(a0, a1, a2)))
    box = (-1, 1, -1, 1)
    sig = 0.15
    f0 = W.finish(W.gaussian_blob(n, n, box, 0.05, 0.1, sig, sig), box,
                  mass=None)
    o.init_conditions(f0)
    o.step(k)
    el = o.get_elements()
    assert np.abs(el[2] - el[5]).max() > 0.02
    f = o.reconstruct_f()
    acc = lambda x: a0 + a1 * x + a2 * x * x
    x = W.site_coords(n, -1, 1)
    rng = np.random.default_rng(12)
    err = 0.0
    for _ in range(400):
        i, j = rng.integers(8, n - 8, size=2)
        q = _dkd_particle(np.array([x[i], x[j]]), -dt, k, acc)
        exact = np.exp(-0.5 * ((q[0] - 0.05) / sig) ** 2
                       - 0.5 * ((q[1] - 0.1) / sig) ** 2)
        err = max(err, abs(f[j, i] - exact))
    assert err < 5e-3, err


def test_det_T_stays_one_under_self_gravity(orc):
    cfg, f0 = W.config("c1_gaussian_256", n=64)
    p = cfg.params()
    p["n_s"] = 0
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    o.step(20)
    d = o.diagnostics()
    assert d["max_det_dev"] < 1e-13
    el = o.get_elements()
    assert np.abs(el[6:]).max() > 0      # curvature did build up


# ---------------------------------------------------- whole-step pins
def _gauss_box(n, sigma=0.1):
    return W.finish(W.gaussian_blob(n, n, (-1, 1, -1, 1), 0.0, 0.0, sigma,
                                    sigma), (-1, 1, -1, 1), 1.0)


def test_free_streaming_conserves_mass_and_follows_closed_form(orc):
    """G = 0: f(x, v, t) = f0(x - v t, v).  Mass is conserved to rounding
    (each row is a uniform shift), and the error against the closed form
    falls like dx^2 (second-order interpolation).  t = 0.19 keeps every row
    shift (j - n/2 + 1/2) t away from a half cell, where the nearest-node
    choice of the six-point stencil flips and the scheme is discontinuous."""
    errs = []
    for n in (64, 128):
        o = orc.Oracle(**box_params(n, 4, dt=0.01, G=0.0, n_s=0))
        f0 = W.gaussian_blob(n, n, (-1, 1, -1, 1), 0.0, 0.0, 0.12, 0.12)
        f0 = W.finish(f0, (-1, 1, -1, 1), mass=None)
        o.init_conditions(f0)
        m0 = o.diagnostics()["mass"]
        o.step(19)
        f = o.reconstruct_f()
        m1 = o.diagnostics()["mass"]
        assert abs(m1 - m0) < 1e-13 * abs(m0)
        x = W.site_coords(n, -1, 1)[None, :]
        v = W.site_coords(n, -1, 1)[:, None]
        t = 0.19
        exact = np.exp(-0.5 * ((x - v * t) / 0.12) ** 2 - 0.5 * (v / 0.12) ** 2)
        errs.append(np.abs(f - exact)[4:-4, 4:-4].max())
    assert errs[0] / errs[1] > 3.0, errs


def test_constant_force_with_remaps_conserves_mass(orc):
    n = 96
    o = orc.Oracle(**box_params(n, 4, dt=0.01, n_s=10,
                                force_mode=orc.FORCE_EXTERNAL,
                                ext=(0.4, 0.0, 0.0)))
    o.init_conditions(_gauss_box(n, 0.08))
    m0 = o.diagnostics()["mass"]
    o.step(30)
    assert o.stepcount == 30 and abs(o.t - 0.3) < 1e-15
    m1 = o.diagnostics()["mass"]
    assert abs(m1 - m0) < 1e-13 * m0


def test_remap_at_t0_is_identity(orc):
    """At t = 0 every element predicts Q = P, so the blended Q_r is P and
    the spline returns F_ini at the nodes (section 2.3.2).  On a power-of-two
    grid every coordinate is exact, so the transport value is exactly F."""
    n = 64
    cfg, f0 = W.config("c2_halos_2048", n=n)
    p = cfg.params()
    p["sx"] = p["sv"] = 4
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    F0 = o.F()
    fr = o.reconstruct_f(orc.SCHEME_REMAP)
    assert np.max(np.abs(fr - F0)) < 1e-13 * np.abs(F0).max()
    ft = o.reconstruct_f(orc.SCHEME_TRANSPORT)
    assert np.array_equal(ft, F0)
    o.remap()
    assert np.max(np.abs(o.F() - F0)) < 1e-13 * np.abs(F0).max()


def test_thermal_sheet_stays_stationary(orc):
    """The self-gravitating isothermal sheet of section 3.2 (rho_S = 4,
    sigma_S = 0.2) is a stationary solution: after ~a third of a dynamical
    time f must stay close to f_ini.  A wrong force sign or factor would
    collapse or expand it by far more."""
    n = 128
    box = (-1, 1, -1, 1)
    f0 = W.finish(W.spitzer_sheet(n, n, box), box, mass=None)
    o = orc.Oracle(**box_params(n, 4, dt=0.01, n_s=25))
    o.init_conditions(f0)
    o.step(100)
    f = o.reconstruct_f()
    dev = np.abs(f - f0).max() / f0.max()
    assert dev < 5e-3, dev


def test_energy_conserved_on_gaussian_run(orc):
    cfg, f0 = W.config("c1_gaussian_256", n=128)
    p = cfg.params()
    p["sx"] = p["sv"] = 4
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    e0 = o.diagnostics()["energy"]
    o.step(100)
    e1 = o.diagnostics()["energy"]
    assert abs(e1 - e0) / abs(e0) < 1e-4


def test_blended_position_is_continuous(orc):
    """Q_r(P) of eq. (interpol) is continuous (section 2.3.2): with W(2d)
    every element outside the beta-restricted set has zero weight, so the
    blend has no jumps when the nearest element or the set changes.  The
    second difference along a fine line stays at the O(h^2) level."""
    n, s = 32, 4
    o = orc.Oracle(**box_params(n, s))
    o.init_conditions(np.ones((n, n)))
    rng = np.random.default_rng(11)
    el = _perturbed_state(o, rng, amp_x=0.05, amp_t=0.02, amp_h=0.05)
    o.set_elements(el)
    for d in ((1.0, 0.0), (0.0, 1.0), (0.6, 0.8)):
        tau = np.linspace(-0.5, 0.5, 8001)
        P = np.stack([0.013 + tau * d[0], -0.021 + tau * d[1]], axis=1)
        Q = o.remap_position(P)
        assert np.isfinite(Q).all()
        d2 = np.abs(Q[2:] - 2 * Q[1:-1] + Q[:-2]).max()
        assert d2 < 1e-6, d2
        # the map stays close to the identity flow it was built from
        assert np.abs(Q - P).max() < 0.1 * (2.0 / n) * s


def test_remap_ignores_diagonals_when_a_three_range_occurs(orc):
    """Section 2.3.2: when either axis needs the full range [-1, 1] the
    diagonal neighbours are left out of the blend (reading R16).  A diagonal
    element moved next to the site would otherwise carry weight."""
    n, s = 32, 4
    o = orc.Oracle(**box_params(n, s))
    o.init_conditions(np.ones((n, n)))
    el = o.get_elements()
    M = n // s
    k, l = 3, 4
    m = l * M + k
    diag = (l + 1) * M + (k + 1)
    dxm = 2.0 / n * s
    P = el[:2, m].copy()
    el[0, diag] = P[0] + 0.3 * dxm
    el[1, diag] = P[1] + 0.3 * dxm
    o.set_elements(el)
    Q = o.remap_position(P[None, :])[0]
    assert np.array_equal(Q, P)


def test_remap_keeps_edge_ring_zero(orc):
    """f = 0 on the outermost sites after every resampling (reading R2)."""
    n = 64
    o = orc.Oracle(**box_params(n, 4, dt=0.01, n_s=5,
                                force_mode=orc.FORCE_EXTERNAL,
                                ext=(3.0, 0.0, 0.0)))
    o.init_conditions(np.ones((n, n)))
    o.step(5)
    F = o.F()
    assert not F[0].any() and not F[-1].any()
    assert not F[:, 0].any() and not F[:, -1].any()
    assert F[1:-1, 1:-1].max() > 0.5


def test_uniform_slab_potential_energy(orc):
    """Potential energy of section 3.2, -1/(4G) int (a^2 - G^2 M^2) dx, for
    a uniform slab of mass M and width L: G M^2 L / 6 (closed form of the
    same integral with a linear a)."""
    n, G, L = 256, 0.7, 1.0
    x = W.site_coords(n, -1, 1)
    v = W.site_coords(n, -1, 1)
    f = np.where(np.abs(x)[None, :] < L / 2, 1.0, 0.0) * \
        np.exp(-0.5 * (v[:, None] / 0.1) ** 2)
    o = orc.Oracle(**box_params(n, 4, G=G))
    o.init_conditions(f)
    d = o.diagnostics()
    M = d["mass"]
    assert abs(d["e_pot"] - G * M * M * L / 6) < 2e-3 * G * M * M * L / 6
    # kinetic energy of a Gaussian velocity profile: M sigma_v^2 / 2
    assert abs(d["e_kin"] - 0.5 * M * 0.01) < 1e-3 * 0.5 * M * 0.01


def test_casimir_entropy_and_norms_of_a_gaussian(orc):
    """Casimir S = -int f ln|f|, L1 = int |f| and L2 = (int f^2)^(1/2) of
    section 3.2 for f = A exp(-(x^2 + v^2) / (2 sigma^2)), mass
    M = 2 pi sigma^2 A: S = M (1 - ln A), L1 = M, L2 = A sigma sqrt(pi)
    (closed forms of the integrals; with sigma = 0.12 the Gaussian's mass
    beyond the box edge is ~1e-15, and the site sums of a Gaussian resolved
    by 15 sites per sigma equal its integral to far below that).  For -f, S changes sign and
    the norms do not, which pins the |f| in the logarithm."""
    n, sig = 256, 0.12
    x = W.site_coords(n, -1, 1)
    r2 = x[None, :] ** 2 + x[:, None] ** 2
    for A in (5.0, 0.2):
        g = A * np.exp(-r2 / (2 * sig * sig))
        M = 2 * math.pi * sig * sig * A
        S = M * (1.0 - math.log(A))
        L2 = A * sig * math.sqrt(math.pi)
        for sign in (1.0, -1.0):
            o = orc.Oracle(**box_params(n, 4))
            o.init_conditions(sign * g)
            d = o.diagnostics()
            assert abs(d["mass"] - sign * M) < 1e-9 * M
            assert abs(d["entropy"] - sign * S) < 1e-9 * abs(S), (A, sign)
            assert abs(d["l1"] - M) < 1e-9 * M
            assert abs(d["l2"] - L2) < 1e-9 * L2
            assert abs(d["e_kin"] - sign * 0.5 * M * sig * sig) < \
                1e-9 * M * sig * sig


# ------------------------------------------------------ paper's numbers
def test_paper_printed_values(orc):
    """Numbers printed in the paper (tests/golden/paper_values.json)."""
    with open(os.path.join(GOLDEN, "paper_values.json")) as fh:
        g = json.load(fh)
    # beta and alpha (section 2.3.3)
    assert abs(orc.BETA_DEFAULT - g["beta"]["value"]) < 5e-4
    assert abs(math.sqrt(3) / 4 - g["alpha"]["value"]) < 5e-3
    assert orc.BETA_DEFAULT <= g["beta_bound"]["value"]
    # thermal sheet: maximum projected density ~ 2 (section 3.2)
    n = 256
    box = (-1, 1, -1, 1)
    sheet = g["sheet"]
    f0 = W.spitzer_sheet(n, n, box, sheet["rho_s"], sheet["sigma_s"])
    o = orc.Oracle(**box_params(n, 4))
    o.init_conditions(f0)
    rho = o.density()
    assert abs(rho.max() - sheet["rho_max"]) < 0.02
    t_dyn = 2 * math.pi / math.sqrt(2 * rho.max())
    assert abs(100.0 / t_dyn - sheet["dyn_times_to_t100"]) < 0.5
    # Gaussian initial condition: total mass ~ 1 (section 3.2)
    gs = g["gaussian"]
    fg = W.gaussian_blob(n, n, box, 0, 0, gs["sigma_g"], gs["sigma_g"],
                         gs["rho_g"])
    o2 = orc.Oracle(**box_params(n, 4))
    o2.init_conditions(fg)
    assert abs(o2.diagnostics()["mass"] - gs["total_mass"]) < 0.01


# ------------------------------------------ E_map (end of section 2.3.3)
def _anharmonic_run(orc, s, n=256, steps=15, **kw):
    box = (-1, 1, -1, 1)
    f0 = W.finish(W.gaussian_blob(n, n, box, 0.05, 0.1, 0.15, 0.15), box,
                  mass=None)
    o = orc.Oracle(**box_params(n, s, dt=0.02, force_mode=orc.FORCE_EXTERNAL,
                                ext=(0.1, -1.3, 2.1), **kw))
    o.init_conditions(f0)
    o.step(steps)
    return o


def test_emap_is_zero_on_a_fresh_lattice(orc):
    """At a reset every element predicts Q = P exactly (T = I, H = 0, and
    P - Q_m is exact on the dyadic grid), so neighbouring predictions
    coincide."""
    cfg, f0 = W.config("c1_gaussian_256", n=64)
    o = orc.Oracle(**box_params(64, 4))
    o.init_conditions(f0)
    assert o.emap() == 0.0


@pytest.mark.parametrize("mode", ["free", "harmonic"])
def test_emap_vanishes_for_linear_flows(orc, mode):
    """A force linear in x makes the map linear: H stays zero, every
    element's expansion is exact, and all predictions of Q agree to
    rounding."""
    box = (-1, 1, -1, 1)
    kw = (dict(G=0.0) if mode == "free" else
          dict(force_mode=orc.FORCE_EXTERNAL, ext=(0.0, -2.0, 0.0)))
    o = orc.Oracle(**box_params(64, 4, dt=0.01, **kw))
    o.init_conditions(W.finish(W.gaussian_blob(64, 64, box, 0, 0, 0.2, 0.2),
                               box, mass=None))
    o.step(25)
    assert not np.any(o.get_elements()[6:])
    assert o.emap() < 1e-12


def test_emap_is_third_order_in_the_element_spacing(orc):
    """Under an anharmonic force neighbouring second-order predictions
    differ by the third-order remainder of the map: halving the element
    spacing on the same grid and flow divides the absolute mismatch
    (E_map x element spacing) by 8."""
    absolute = []
    for s in (16, 8, 4):
        o = _anharmonic_run(orc, s)
        absolute.append(o.emap() * s * (2.0 / 256))
    for a, b in zip(absolute, absolute[1:]):
        assert 2.8 < math.log2(a / b) < 3.2, absolute


def test_adaptive_remap_follows_the_threshold(orc):
    """With adaptive resampling, a check after step 5 remaps (fresh T = I)
    exactly when E_map of that state exceeds the threshold."""
    ref = _anharmonic_run(orc, 8, n=128, steps=5)
    e5 = ref.emap()
    assert e5 > 0.0
    for thr, expect_remap in ((0.5 * e5, True), (2.0 * e5, False)):
        o = _anharmonic_run(orc, 8, n=128, steps=5, emap_max=thr,
                            emap_every=5)
        el = o.get_elements()
        fresh = np.all(el[2] == 1.0) and np.all(el[5] == 1.0) and \
            not np.any(el[3]) and not np.any(el[4])
        assert fresh == expect_remap, (thr, e5)
    # checks at other steps only
    o = _anharmonic_run(orc, 8, n=128, steps=5, emap_max=0.5 * e5,
                        emap_every=3)
    assert not np.all(o.get_elements()[2] == 1.0)
