"""Variable time step (section 2.4, dt <= C_dyn / sqrt(rho_max)) on the GPU
against the oracle.

The step sizes and the time live in a device clock that the element pass
updates from the density it builds the force from, so no step waits for the
host.  In FP64 the density maximum, the bound and every step size are the
oracle's to the rounding of the density sums (tests/parity.py), so a
variable-step run follows the oracle's trajectory through each element-pass
variant: the shared field (small grids), the field rebuilt per workgroup
(few elements, many columns) and the separate field kernel (more than 2048
columns)."""
import math

import numpy as np
import pytest

import workloads as W
from parity import RTOL, TIME_RTOL, assert_elements_close

pytestmark = pytest.mark.gpu


def close_t(a, b):
    return abs(a - b) <= TIME_RTOL * abs(b)


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def halos(nx, nv, seed=7, k=3):
    rng = np.random.default_rng(seed)
    box = (-1.0, 1.0, -1.0, 1.0)
    return W.finish(W.halo_sum(nx, nv, box, rng, k), box, 1.0)


def bound_c(f0, nv, frac):
    """C_dyn that makes the first step frac x the cap of 1."""
    g = np.array(f0, dtype=np.float64)
    g[0, :] = g[-1, :] = 0.0
    g[:, 0] = g[:, -1] = 0.0
    return frac * math.sqrt((2.0 / nv * g.sum(axis=0)).max())


def pair(vp, orc, p, f0, precision="fp64"):
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    g = vp.VlasovRun(device="cuda:0", precision=precision, **p)
    g.init_conditions(f0)
    return o, g


@pytest.mark.parametrize("nx,nv,s,steps,n_s,path", [
    (128, 128, 8, 24, 10, "shared field"),
    (2048, 32, 8, 12, 5, "field per workgroup"),
    (2304, 32, 8, 12, 5, "separate field kernel"),
    # 64 x 16 patches: the element pass claims slots through workgroup tables
    (4096, 1024, 4, 6, 3, "separate field kernel, tables"),
])
def test_fp64_variable_step_matches_oracle(vp, orc, nx, nv, s, steps, n_s,
                                           path):
    f0 = halos(nx, nv)
    cap = 0.02
    p = dict(nx=nx, nv=nv, sx=s, dt=cap, n_s=n_s,
             c_dyn=cap * bound_c(f0, nv, 0.6))
    print(f"[{path}] nx={nx} nv={nv} s={s} steps={steps}", flush=True)
    o, g = pair(vp, orc, p, f0)
    d0 = g.diagnostics()
    assert close_t(d0["dt"], o.dt) and d0["t"] == 0.0 and o.dt < cap
    # a second engine run takes the steps one call at a time: the element
    # pass then ends each step without the next predictor
    g1 = vp.VlasovRun(device="cuda:0", **p)
    g1.init_conditions(f0)
    dts = set()
    for _ in range(steps):
        o.step(1)
        g1.step(1)
        dts.add(o.dt)
    assert len(dts) > 2
    g.step(steps)
    for run in (g, g1):
        d = run.diagnostics()
        assert close_t(d["t"], o.t) and close_t(d["dt"], o.dt)
        assert d["step"] == steps
        t, st = run.time()
        assert t == d["t"] and st == steps
        assert_elements_close(run.get_elements().cpu().numpy(), o)
    f_ref = o.reconstruct_f()
    f = g.reconstruct_f().cpu().numpy()
    assert np.abs(f - f_ref).max() <= RTOL * np.abs(f_ref).max()
    g.sync()
    g1.sync()


def test_variable_step_with_emap_resampling(vp, orc):
    """Both adaptive options at once: the step from the density bound and
    resampling when E_map exceeds a threshold (checked every 4 steps)."""
    n = 128
    f0 = halos(n, n, seed=9)
    cap = 0.01
    p = dict(nx=n, sx=8, dt=cap, n_s=0, c_dyn=cap * bound_c(f0, n, 0.7))
    probe = orc.Oracle(**p)
    probe.init_conditions(f0)
    probe.step(8)
    p.update(emap_max=0.5 * probe.emap(), emap_every=4)
    o, g = pair(vp, orc, p, f0)
    o.step(24)
    g.step(24)
    free = orc.Oracle(**dict(p, emap_max=0.0, emap_every=0))
    free.init_conditions(f0)
    free.step(24)
    assert not np.array_equal(free.get_elements(), o.get_elements())
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    d = g.diagnostics()
    assert close_t(d["t"], o.t) and close_t(d["dt"], o.dt)
    g.sync()


def test_mixed_variable_step_tracks_oracle(vp, orc):
    n, s = 256, 8
    f0 = halos(n, n, seed=11)
    cap = 0.02
    p = dict(nx=n, sx=s, dt=cap, n_s=10, c_dyn=cap * bound_c(f0, n, 0.5))
    o, g = pair(vp, orc, p, f0, "mixed")
    o.step(25)
    g.step(25)
    d = g.diagnostics()
    # the steps come from a density summed from FP32 f: rho_max carries at
    # most the 1e-5 relative error allowed on f, dt half of it (square
    # root), and t, a sum of positive steps, no more than dt
    assert abs(d["t"] - o.t) <= 5e-6 * o.t
    f_ref = o.reconstruct_f()
    f = g.reconstruct_f().cpu().numpy().astype(np.float64)
    assert np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref) <= 1e-5
    g.sync()


def test_unbinding_bound_equals_fixed_step_run(vp):
    n = 128
    f0 = halos(n, n, seed=5)
    base = dict(nx=n, sx=8, dt=0.01, n_s=7)
    a = vp.VlasovRun(device="cuda:0", **base)
    b = vp.VlasovRun(device="cuda:0", c_dyn=1e3, **base)
    a.init_conditions(f0)
    b.init_conditions(f0)
    a.step(15)
    b.step(15)
    assert np.array_equal(a.get_elements().cpu().numpy(),
                          b.get_elements().cpu().numpy())
    assert np.array_equal(a.reconstruct_f().cpu().numpy(),
                          b.reconstruct_f().cpu().numpy())
    d = b.diagnostics()
    assert d["dt"] == 0.01 and d["t"] == pytest.approx(0.15, rel=1e-14)
    a.sync()
    b.sync()


def test_variable_step_validation(vp):
    import torch
    with pytest.raises(vp.VPError):
        vp.VlasovRun(device="cuda:0", nx=64, sx=8, dt=0.01,
                     force_mode=vp.FORCE_EXTERNAL, c_dyn=0.1)
    with pytest.raises(vp.VPError):
        vp.VlasovRun(device="cuda:0", nx=64, sx=8, dt=0.01, c_dyn=-1.0)
    n = 64
    f0 = torch.as_tensor(halos(n, n), device="cuda:0")
    out = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    srv = vp.Server(precision="fp64", max_active=2, pool_bytes=1 << 26)
    res, st = srv.run([dict(params=dict(nx=n, sx=4, dt=1e-3, n_s=10,
                                        precision="fp64", c_dyn=0.01),
                            f0=f0, out=out, nsteps=3, tag=1,
                            arrival_s=0.0)])
    assert res[0]["status"] == vp.EINVAL and st["completed"] == 1
    srv.close()
