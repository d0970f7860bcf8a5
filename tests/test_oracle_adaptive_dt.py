"""Pins of the oracle's variable time step (section 2.4: dt <= C_dyn /
sqrt(rho_max), rho the projected density), each against something other
than the oracle's own formula:

* the first step against the bound evaluated on the initial condition by
  numpy (an independent density sum);
* free streaming (G = 0) with a step that varies from step to step: every
  element must sit at Q + v t and carry T_xv = t, t the sum of the steps,
  which fixes the half-step bookkeeping of the predictor and corrector;
* the scaling symmetry x -> 4 x, f -> f / 4, G -> G / 4, C_dyn -> 2 C_dyn of
  the Vlasov-Poisson system: rho -> rho / 4, so the bound gives dt -> 4 dt
  only with the exponent 1/2; every operation then scales by a power of
  two and the runs agree bit for bit;
* a bound that never binds reproduces the fixed-step run exactly.
"""
import math

import numpy as np
import pytest

import workloads as W

BOX = (-1.0, 1.0, -1.0, 1.0)


def halos(n, seed=7, k=3, box=BOX):
    rng = np.random.default_rng(seed)
    return W.finish(W.halo_sum(n, n, box, rng, k), box, 1.0)


def edge_zeroed(f):
    g = np.array(f, dtype=np.float64)
    g[0, :] = g[-1, :] = 0.0
    g[:, 0] = g[:, -1] = 0.0
    return g


def test_first_step_obeys_initial_density_bound(orc):
    n = 64
    f0 = halos(n)
    dv = 2.0 / n
    rho_max = (dv * edge_zeroed(f0).sum(axis=0)).max()
    C = 0.02
    o = orc.Oracle(nx=n, sx=8, dt=0.05, n_s=0, c_dyn=C)
    o.init_conditions(f0)
    assert o.dt == pytest.approx(C / math.sqrt(rho_max), rel=1e-14)
    assert o.dt < 0.05
    # a bound above the cap leaves the nominal step
    o2 = orc.Oracle(nx=n, sx=8, dt=0.05, n_s=0, c_dyn=10.0)
    o2.init_conditions(f0)
    assert o2.dt == 0.05
    # no positive density: the cap
    o3 = orc.Oracle(nx=n, sx=8, dt=0.05, n_s=0, c_dyn=C)
    o3.init_conditions(np.zeros((n, n)))
    assert o3.dt == 0.05


def test_variable_step_free_streaming(orc):
    n = 64
    f0 = halos(n)
    rho0 = (2.0 / n * edge_zeroed(f0).sum(axis=0)).max()
    cap = 0.05
    p = dict(nx=n, sx=8, dt=cap, n_s=0, G=0.0, c_dyn=0.5 * cap * math.sqrt(rho0))
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    q = o.get_elements()
    dts = [o.dt]
    for _ in range(30):
        o.step(1)
        dts.append(o.dt)
    # the halos shear apart, rho_max falls and the step grows
    assert max(dts) / min(dts) > 1.1 and max(dts) <= cap
    t = o.t
    el = o.get_elements()
    scale = np.abs(q[0]).max() + np.abs(q[1]).max() * t
    assert np.abs(el[0] - (q[0] + q[1] * t)).max() <= 1e-14 * scale
    assert np.array_equal(el[1], q[1])
    assert np.abs(el[3] - t).max() <= 1e-14 * t
    assert np.all(el[2] == 1.0) and np.all(el[5] == 1.0) and not np.any(el[4])


@pytest.mark.parametrize("n_s", [0, 6])
def test_scaling_symmetry_fixes_the_exponent(orc, n_s):
    n, steps = 48, 14
    f0 = halos(n, seed=3)
    C = 0.03
    pa = dict(nx=n, sx=8, dt=0.04, n_s=n_s, G=1.0, c_dyn=C)
    pb = dict(pa, x_min=-4.0, x_max=4.0, G=0.25, c_dyn=2.0 * C, dt=0.16)
    a = orc.Oracle(**pa)
    a.init_conditions(f0)
    b = orc.Oracle(**pb)
    b.init_conditions(f0 / 4.0)
    assert b.dt == 4.0 * a.dt and a.dt < 0.04
    seen = set()
    for _ in range(steps):
        a.step(1)
        b.step(1)
        seen.add(a.dt)
        assert b.dt == 4.0 * a.dt
        assert b.t == 4.0 * a.t
    assert len(seen) > 3  # the step really varied
    ea, eb = a.get_elements(), b.get_elements()
    # x, T_x., H scale with the powers of 4 of their x factors
    powers = [1, 0, 0, 1, -1, 0, -1, 0, 1, -2, -1, 0]
    for k, pw in enumerate(powers):
        assert np.array_equal(eb[k], ea[k] * 4.0 ** pw), k
    assert np.array_equal(b.reconstruct_f(), a.reconstruct_f() / 4.0)


def test_unbinding_bound_equals_fixed_step(orc):
    n = 48
    f0 = halos(n, seed=5)
    base = dict(nx=n, sx=8, dt=0.01, n_s=5, G=1.0)
    a = orc.Oracle(**base)
    b = orc.Oracle(**dict(base, c_dyn=1e3))
    a.init_conditions(f0)
    b.init_conditions(f0)
    a.step(12)
    b.step(12)
    assert np.array_equal(a.get_elements(), b.get_elements())
    assert np.array_equal(a.reconstruct_f(), b.reconstruct_f())
    assert b.t == pytest.approx(a.t, rel=1e-14) and b.dt == 0.01


def test_rejects_variable_step_with_external_force(orc):
    with pytest.raises(orc.OracleError):
        orc.Oracle(nx=32, sx=8, dt=0.01, force_mode=orc.FORCE_EXTERNAL,
                   c_dyn=0.1)
