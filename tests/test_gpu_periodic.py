"""Periodic-x variant (plasma for G < 0, periodic gravity for G > 0) on the
GPU against the oracle.

The FP64 engine follows the oracle to the rounding of its density sums
(rules in tests/parity.py): elements re-enter the box after each drift,
sites see elements through their nearest image (the block lists wrap at the
seam), lattice neighbours wrap with a one-period shift, F_ini and the spline
repeat in x (ghost columns), the cyclic spline system rounds the same way.
Cases cover the three element-pass variants, the seam blocks, small rings
whose elements are all too wide for lists, the variable step and E_map on a
ring."""
import math

import numpy as np
import pytest

from parity import (RTOL, TIME_RTOL, assert_elements_close,
                    assignment_same_state, force_close, rel_linf)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def ring(nx, nv, k_modes, alpha, seed=0):
    """Maxwellian plasma / gas on one period with a few seeded Fourier
    perturbations of the density (mean density 1)."""
    rng = np.random.default_rng(seed)
    L = 4.0 * math.pi
    x = (np.arange(nx) + 0.5) * L / nx
    v = -6.0 + (np.arange(nv) + 0.5) * 12.0 / nv
    X, V = np.meshgrid(x, v)
    pert = np.ones_like(X)
    for m in k_modes:
        pert += alpha * rng.uniform(0.5, 1.0) * np.cos(
            2.0 * math.pi * m * X / L + rng.uniform(0, 2 * math.pi))
    # a drifting beam makes the flow cross the seam in both directions
    f0 = pert * (0.8 * np.exp(-0.5 * V * V) + 0.2 * np.exp(
        -0.5 * ((V - 2.0) / 0.5) ** 2) / 0.5) / math.sqrt(2.0 * math.pi)
    return L, f0


def params(nx, nv, L, s, G, dt, n_s, **kw):
    p = dict(nx=nx, nv=nv, x_min=0.0, x_max=L, v_min=-6.0, v_max=6.0, sx=s,
             sv=s, G=G, dt=dt, n_s=n_s, bc=1)
    p.update(kw)
    return p


def pair(vp, orc, p, f0, precision="fp64"):
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    g = vp.VlasovRun(device="cuda:0", precision=precision, **p)
    g.init_conditions(f0)
    return o, g


@pytest.mark.parametrize("nx,nv,s,G,steps,n_s,path", [
    (64, 128, 4, -0.5, 27, 10, "plasma, shared field"),
    (128, 64, 8, 0.25, 21, 8, "gravity, shared field"),
    (2048, 32, 8, -0.5, 10, 4, "plasma, field per workgroup"),
    (2304, 32, 8, -0.5, 10, 4, "plasma, separate field kernel"),
    # 64 x 16 patches of 16 x 16 elements: slot claims through the
    # workgroup tables, whose keys take unwrapped block columns at the seam
    (4096, 1024, 4, -0.5, 6, 4, "plasma, separate field kernel, tables"),
])
def test_fp64_periodic_matches_oracle(vp, orc, nx, nv, s, G, steps, n_s,
                                      path):
    L, f0 = ring(nx, nv, (1, 2, 3), 0.05, seed=nx)
    p = params(nx, nv, L, s, G, 0.1, n_s)
    print(f"[{path}] nx={nx} nv={nv} s={s} steps={steps}", flush=True)
    o, g = pair(vp, orc, p, f0)
    assert np.array_equal(g.assignment().cpu().numpy(), o.assignment(False))
    o.step(steps)
    g.step(steps)
    el = g.get_elements().cpu().numpy()
    assert_elements_close(el, o)
    assert np.all((el[0] >= 0.0) & (el[0] < L))
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    assert rel_linf(g.density().cpu().numpy(), o.density()) <= RTOL
    fr = g.reconstruct_f(vp.SCHEME_REMAP).cpu().numpy()
    assert rel_linf(fr, o.reconstruct_f(1)) <= RTOL
    # sites next to the seam are served by elements from the other end
    a, a_ref = assignment_same_state(g, o)
    assert np.array_equal(a, a_ref)
    near = a[:, 0][a[:, 0] >= 0]
    assert np.any(o.get_elements()[0][near] > 0.5 * L)
    g.sync()


def test_periodic_force_matches_oracle(vp, orc):
    nx, L = 256, 4.0 * math.pi
    rng = np.random.default_rng(3)
    rho = 1.0 + 0.3 * rng.uniform(-1, 1, nx)
    o = orc.Oracle(**params(nx, 32, L, 8, -0.5, 0.1, 0))
    g = vp.VlasovRun(device="cuda:0", **params(nx, 32, L, 8, -0.5, 0.1, 0))
    force_close([t.cpu().numpy() for t in g.poisson(rho)], o.poisson(rho),
                rho, o)
    g.sync()


@pytest.mark.parametrize("nx,s", [(8, 4), (16, 8), (24, 4)])
def test_small_rings_full_scan(vp, orc, nx, s):
    """Rings too short for nearest-image lists: every query scans all
    elements."""
    L, f0 = ring(nx, 32, (1,), 0.1, seed=nx)
    p = params(nx, 32, L, s, -0.5, 0.1, 5)
    o, g = pair(vp, orc, p, f0)
    o.step(12)
    g.step(12)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    g.sync()


def test_periodic_variable_step_and_emap(vp, orc):
    nx, nv, s = 128, 64, 8
    L, f0 = ring(nx, nv, (1, 2), 0.1, seed=5)
    p = params(nx, nv, L, s, 0.25, 0.1, 0, c_dyn=0.05)
    probe = orc.Oracle(**p)
    probe.init_conditions(f0)
    probe.step(6)
    p.update(emap_max=0.5 * probe.emap(), emap_every=3)
    o, g = pair(vp, orc, p, f0)
    o.step(18)
    g.step(18)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    d = g.diagnostics()
    assert abs(d["t"] - o.t) <= TIME_RTOL * o.t
    assert abs(d["dt"] - o.dt) <= TIME_RTOL * o.dt
    # E_map of one element state is a maximum of per-site values computed
    # with the same operations: exact for the oracle's state
    g.set_elements(o.get_elements())
    d = g.diagnostics()
    assert d["emap"] == o.emap()
    ref = o.diagnostics()
    for k in ("mass", "e_kin", "e_pot", "energy"):
        assert abs(d[k] - ref[k]) <= 1e-11 * max(1.0, abs(ref[k])), k
    g.sync()


def test_mixed_periodic_tracks_oracle(vp, orc):
    nx, nv, s = 256, 128, 8
    L, f0 = ring(nx, nv, (1, 2, 3), 0.05, seed=9)
    p = params(nx, nv, L, s, -0.5, 0.1, 10)
    o, g = pair(vp, orc, p, f0, "mixed")
    o.step(25)
    g.step(25)
    f_ref = o.reconstruct_f()
    f = g.reconstruct_f().cpu().numpy().astype(np.float64)
    assert np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref) <= 1e-5
    g.sync()


def test_landau_damping_on_gpu(vp):
    """The plasma test of the oracle pins, run by the engine: field energy
    of the k = 0.5 mode damps at the kinetic rate (-0.1534)."""
    import torch
    k, nx, nv = 0.5, 64, 128
    L = 2.0 * math.pi / k
    x = (np.arange(nx) + 0.5) * L / nx
    v = -6.0 + (np.arange(nv) + 0.5) * 12.0 / nv
    X, V = np.meshgrid(x, v)
    f0 = (1.0 + 0.01 * np.cos(k * X)) * np.exp(-0.5 * V * V) / math.sqrt(
        2.0 * math.pi)
    g = vp.VlasovRun(device="cuda:0", **params(nx, nv, L, 4, -0.5, 0.1, 10))
    g.init_conditions(torch.as_tensor(f0, device="cuda:0"))
    ts, W = [], []
    for _ in range(230):
        g.step(1)
        d = g.diagnostics()
        ts.append(d["t"])
        W.append(d["e_pot"])
    ts, W = np.array(ts), np.array(W)
    pk = [i for i in range(1, len(W) - 1) if W[i] > W[i - 1] and W[i] >= W[i + 1]]
    tp, wp = ts[pk], W[pk]
    sel = (tp > 1.0) & (tp < 22.0)
    gamma = np.polyfit(tp[sel], np.log(wp[sel]), 1)[0] / 2.0
    assert abs(gamma + 0.15336) <= 0.02 * 0.15336, gamma
    g.sync()


def test_periodic_validation(vp):
    import torch
    with pytest.raises(vp.VPError):  # nx not a multiple of 8
        vp.VlasovRun(device="cuda:0", **params(36, 32, 1.0, 4, -0.5, 0.1, 0))
    with pytest.raises(vp.VPError):  # external force
        vp.VlasovRun(device="cuda:0", **params(64, 32, 1.0, 4, -0.5, 0.1, 0,
                                               force_mode=1))
    n = 64
    f0 = torch.zeros((n, n), dtype=torch.float64, device="cuda:0")
    out = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    srv = vp.Server(precision="fp64", max_active=2, pool_bytes=1 << 26)
    res, st = srv.run([dict(params=dict(nx=n, sx=4, dt=1e-3, n_s=10,
                                        precision="fp64", bc=1),
                            f0=f0, out=out, nsteps=3, tag=1,
                            arrival_s=0.0)])
    assert res[0]["status"] == vp.EINVAL and st["completed"] == 1
    srv.close()
