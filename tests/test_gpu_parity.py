"""Parity of the HIP engine (through the C ABI) with the CPU oracle.

The FP64 engine must give the oracle's nearest-element assignment bit for bit
for the same element state, and f, rho to relative L-inf 1e-12 (max |diff| /
max |oracle|); element states along a self-gravitating trajectory, and the
force of a given density, agree to the rounding of the density sums (rules
in tests/parity.py).  Inputs are seeded and synthetic; element states are
injected into both sides from the same seeded arrays.
"""
import numpy as np
import pytest

import workloads as W
from parity import (RTOL, assert_elements_close, assignment_same_state,
                    force_close, rel_linf)

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def params(n, s, nv=None, sv=None, **kw):
    p = dict(nx=n, nv=nv or n, sx=s, sv=sv or s, dt=kw.pop("dt", 1e-3),
             G=kw.pop("G", 1.0), n_s=kw.pop("n_s", 0))
    p.update(kw)
    return p


def pair(vp, orc, p, f0, precision="fp64"):
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    g = vp.VlasovRun(device="cuda:0", precision=precision, **p)
    g.init_conditions(f0)
    return o, g


def perturbed(o, seed, amp_x=0.3, amp_t=0.15, amp_h=2.0):
    rng = np.random.default_rng(seed)
    el = o.get_elements()
    E = el.shape[1]
    dxm = (2.0 / o.nx) * o.sx
    dvm = (2.0 / o.nv) * o.sv
    el[0] += rng.uniform(-amp_x, amp_x, E) * dxm
    el[1] += rng.uniform(-amp_x, amp_x, E) * dvm
    for r in (2, 3, 4, 5):
        el[r] += rng.uniform(-amp_t, amp_t, E)
    el[6:] = rng.uniform(-amp_h, amp_h, (6, E))
    return el


def halos(n, nv=None, seed=7, k=3):
    nv = nv or n
    rng = np.random.default_rng(seed)
    box = (-1.0, 1.0, -1.0, 1.0)
    return W.finish(W.halo_sum(n, nv, box, rng, k), box, 1.0)


GRIDS = [(64, 4, 64, 4), (64, 8, 48, 8), (60, 4, 40, 2), (96, 16, 64, 16),
         (40, 2, 40, 5), (32, 1, 24, 3)]


@pytest.mark.parametrize("n,s,nv,sv", GRIDS)
def test_assignment_and_transport_bitexact(vp, orc, n, s, nv, sv):
    p = params(n, s, nv, sv)
    f0 = halos(n, nv)
    o, g = pair(vp, orc, p, f0)
    for trial, seed in enumerate((0, 11, 12)):
        if trial:
            el = perturbed(o, seed + n)
            o.set_elements(el)
            g.set_elements(el)
        a_ref = o.assignment(brute=True)
        a_gpu = g.assignment().cpu().numpy()
        assert np.array_equal(a_gpu, a_ref), (trial,
                                              int((a_gpu != a_ref).sum()))
        f_ref = o.reconstruct_f(orc.SCHEME_TRANSPORT)
        f_gpu = g.reconstruct_f(vp.SCHEME_TRANSPORT).cpu().numpy()
        assert rel_linf(f_gpu, f_ref) <= RTOL
        fr_ref = o.reconstruct_f(orc.SCHEME_REMAP)
        fr_gpu = g.reconstruct_f(vp.SCHEME_REMAP).cpu().numpy()
        assert rel_linf(fr_gpu, fr_ref) <= RTOL
    g.sync()


def test_density_and_poisson(vp, orc):
    p = params(128, 8)
    o, g = pair(vp, orc, p, halos(128))
    el = perturbed(o, 5, amp_x=0.1, amp_t=0.05, amp_h=0.5)
    o.set_elements(el)
    g.set_elements(el)
    r_ref = o.density()
    r_gpu = g.density().cpu().numpy()
    assert rel_linf(r_gpu, r_ref) <= RTOL
    a_ref = o.poisson(r_ref)
    a_gpu = [t.cpu().numpy() for t in g.poisson(r_ref)]
    force_close(a_gpu, a_ref, r_ref, o)
    g.sync()


@pytest.mark.parametrize("nx", [2304, 4100])
def test_density_and_poisson_wide_grids(vp, orc, nx):
    """Above 2048 columns the field runs as two launches: column sums and
    chunk prefixes, then the carries, M_left and a, a', a'' spread over the
    workgroups (4100 columns leave a ragged last workgroup of 4 columns).
    Density from a perturbed element state and the force of a given rho,
    both against the oracle."""
    p = params(nx, 4, nv=32)
    o, g = pair(vp, orc, p, halos(nx, 32, seed=nx))
    el = perturbed(o, 9, amp_x=0.1, amp_t=0.05, amp_h=0.5)
    o.set_elements(el)
    g.set_elements(el)
    print(f"[wide field] nx={nx}", flush=True)
    r_ref = o.density()
    assert rel_linf(g.density().cpu().numpy(), r_ref) <= RTOL
    rho = np.random.default_rng(nx).uniform(0.0, 2.0, nx)
    force_close([t.cpu().numpy() for t in g.poisson(rho)], o.poisson(rho),
                rho, o)
    g.sync()


@pytest.mark.parametrize("nx,nv,sx,sv", [(4104, 4096, 8, 8),
                                         (4096, 2056, 4, 8)])
def test_registration_through_workgroup_tables(vp, orc, nx, nv, sx, sv):
    """Element passes over many patches of 16 x 16 elements with strides up
    to 8 register their slot claims through a table per workgroup (one
    device atomic per block and workgroup).  4104 x 4096 sites, s = 8:
    33 x 32 patches, the last column of patches 1 element wide; T is
    perturbed by up to 0.3, so windows reach ~13 sites and boxes up to
    5 x 5 blocks, past the 16 the table takes (the rest claim directly).
    4096 x 2056 sites with strides 4 along x and 8 along v: 64 x 17
    patches, the last row of patches 1 element high.  The assignment of
    the injected state, then the elements and f after two steps (the
    separate field kernel: more than 2048 columns), against the oracle."""
    p = params(nx, sx, nv=nv, sv=sv)
    print(f"[table registration] {nx}x{nv} sx={sx} sv={sv}", flush=True)
    o, g = pair(vp, orc, p, halos(nx, nv, seed=nx))
    el = perturbed(o, 21, amp_x=0.3, amp_t=0.3, amp_h=0.5)
    o.set_elements(el)
    g.set_elements(el)
    a_gpu = g.assignment().cpu().numpy()
    assert np.array_equal(a_gpu, o.assignment())
    o.step(2)
    g.step(2)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    g.sync()


@pytest.mark.parametrize("mode", ["free", "constant", "harmonic",
                                  "anharmonic"])
def test_element_motion_matches_oracle(vp, orc, mode):
    ext = {"free": None, "constant": (0.4, 0.0, 0.0),
           "harmonic": (0.0, -2.0, 0.0), "anharmonic": (0.1, -1.3, 2.1)}[mode]
    p = params(64, 4, dt=0.01, n_s=0)
    if ext is None:
        p["G"] = 0.0
    else:
        p.update(force_mode=1, ext=ext)
    o, g = pair(vp, orc, p, halos(64))
    o.step(17)
    g.step(17)
    # no density sum enters these forces (G = 0 or an external field): the
    # element states agree bit for bit
    el_ref = o.get_elements()
    el_gpu = g.get_elements().cpu().numpy()
    assert np.array_equal(el_gpu, el_ref)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    g.sync()


def test_full_run_c1_fp64(vp, orc):
    """Config 0: 256^2 Gaussian, s = 4, 200 steps, remap every 25."""
    cfg, f0 = W.config("c1_gaussian_256")
    p = params(cfg.n, cfg.s, dt=cfg.dt, n_s=cfg.n_s)
    o, g = pair(vp, orc, p, f0)
    o.step(cfg.steps)
    g.step(cfg.steps)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    assert rel_linf(g.density().cpu().numpy(), o.density()) <= RTOL
    d_ref = o.diagnostics()
    d_gpu = g.diagnostics()
    for k in ("mass", "e_kin", "e_pot", "entropy", "l1", "l2"):
        assert abs(d_gpu[k] - d_ref[k]) <= 1e-10 * abs(d_ref[k]), k
    assert d_gpu["max_det_dev"] < 1e-13
    assert d_gpu["step"] == cfg.steps


def test_halo_run_with_remaps(vp, orc):
    """Config 1 recipe at 512^2 (s = 8): 120 steps, remap every 50."""
    cfg, f0 = W.config("c2_halos_2048", n=512)
    p = params(512, 8, dt=cfg.dt, n_s=50)
    o, g = pair(vp, orc, p, f0)
    o.step(120)
    g.step(120)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    assert rel_linf(g.density().cpu().numpy(), o.density()) <= RTOL
    a_gpu, a_ref = assignment_same_state(g, o)
    assert np.array_equal(a_gpu, a_ref)
    g.sync()


def test_list_overflow_falls_back_to_full_scan(vp, orc):
    """All elements piled into a few blocks overflow the block lists; the
    full scan keeps the assignment exact."""
    p = params(64, 4)
    o, g = pair(vp, orc, p, halos(64))
    el = o.get_elements()
    rng = np.random.default_rng(3)
    E = el.shape[1]
    el[0] = rng.uniform(-0.05, 0.05, E)
    el[1] = rng.uniform(-0.05, 0.05, E)
    o.set_elements(el)
    g.set_elements(el)
    assert np.array_equal(g.assignment().cpu().numpy(), o.assignment(True))
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    assert g.diagnostics()["overflow_blocks"] > 0


def test_wide_element_forces_full_scan(vp, orc):
    p = params(64, 4)
    o, g = pair(vp, orc, p, halos(64))
    el = o.get_elements()
    el[3, 5] = 400.0     # a huge shear: the window spans the whole box
    o.set_elements(el)
    g.set_elements(el)
    assert np.array_equal(g.assignment().cpu().numpy(), o.assignment(True))
    g.sync()


def test_numeric_error_reported(vp, orc):
    p = params(32, 4)
    o, g = pair(vp, orc, p, halos(32))
    el = o.get_elements()
    el[2, 3] = 0.0       # det T = 0
    el[5, 3] = 0.0
    g.set_elements(el)
    g.step(1)
    with pytest.raises(vp.VPError) as ei:
        g.sync()
    assert ei.value.code == vp.ENUMERIC


def test_host_f0_upload_matches_device(vp, orc):
    import ctypes as C
    p = params(48, 4)
    f0 = halos(48)
    g1 = vp.VlasovRun(device="cuda:0", **p)
    g1.init_conditions(f0)
    g2 = vp.VlasovRun(device="cuda:0", **p)
    f0c = np.ascontiguousarray(f0)
    rc = vp.lib().vp_init_conditions(
        g2.h, f0c.ctypes.data_as(C.c_void_p), 0)
    assert rc == 0
    a = g1.reconstruct_f(vp.SCHEME_REMAP).cpu().numpy()
    b = g2.reconstruct_f(vp.SCHEME_REMAP).cpu().numpy()
    assert np.array_equal(a, b)


def test_mixed_precision_against_fp64_oracle(vp, orc):
    """FP32 f / interpolation, FP64 elements and force: relative L2 on f
    within 1e-5 of the FP64 oracle and the same energy drift to 1e-6."""
    cfg, f0 = W.config("c1_gaussian_256")
    p = params(cfg.n, cfg.s, dt=cfg.dt, n_s=cfg.n_s)
    o, g = pair(vp, orc, p, f0, precision="mixed")
    e0_ref = o.diagnostics()["energy"]
    e0_gpu = g.diagnostics()["energy"]
    o.step(cfg.steps)
    g.step(cfg.steps)
    f_ref = o.reconstruct_f()
    f_gpu = g.reconstruct_f().cpu().numpy().astype(np.float64)
    l2 = np.linalg.norm(f_gpu - f_ref) / np.linalg.norm(f_ref)
    assert l2 <= 1e-5, l2
    d_ref = o.diagnostics()["energy"]
    d_gpu = g.diagnostics()["energy"]
    drift_ref = (d_ref - e0_ref) / abs(e0_ref)
    drift_gpu = (d_gpu - e0_gpu) / abs(e0_gpu)
    assert abs(drift_gpu - drift_ref) <= 1e-6, (drift_gpu, drift_ref)


def test_reads_right_after_a_resampling(vp, orc):
    """The spline fit that follows a resampling inside a step overlaps the
    next steps; every reader of the new coefficients waits for it: the remap
    reconstruction called at once, the next resampling a few steps later, a
    new initial condition given right after one (its host upload is staged
    through the coefficient buffer)."""
    f0 = halos(256, seed=11)
    p = params(256, 4, dt=1e-3, n_s=4)
    o, g = pair(vp, orc, p, f0)
    o.step(4)
    g.step(4)
    assert rel_linf(g.reconstruct_f(1).cpu().numpy(), o.reconstruct_f(1)) <= RTOL
    o.step(4)
    g.step(4)
    assert_elements_close(g.get_elements().cpu().numpy(), o)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    import ctypes as C
    f1 = np.ascontiguousarray(halos(256, seed=12))
    o.step(4)
    g.step(4)
    o.init_conditions(f1)
    assert vp.lib().vp_init_conditions(
        g.h, f1.ctypes.data_as(C.c_void_p), 0) == 0
    o.step(5)
    g.step(5)
    assert rel_linf(g.reconstruct_f().cpu().numpy(), o.reconstruct_f()) <= RTOL
    assert rel_linf(g.reconstruct_f(1).cpu().numpy(), o.reconstruct_f(1)) <= RTOL
    g.sync()


def test_contexts_are_independent(vp, orc):
    """Two runs on two streams, their steps interleaved (and one of them
    resampling while the other steps), give bit for bit what each gives
    alone: a context keeps all its state in its own workspace."""
    import torch
    fa, fb = halos(128, seed=21), halos(96, nv=64, seed=22)
    pa = params(128, 4, dt=1e-3, n_s=6)
    pb = params(96, 8, nv=64, sv=4, dt=2e-3, n_s=5)

    def alone(p, f):
        g = vp.VlasovRun(device="cuda:0", **p)
        g.init_conditions(f)
        g.step(13)
        out = (g.get_elements().cpu().numpy(), g.reconstruct_f().cpu().numpy())
        g.sync()
        return out

    ref_a, ref_b = alone(pa, fa), alone(pb, fb)
    sa, sb = torch.cuda.Stream(), torch.cuda.Stream()
    ga = vp.VlasovRun(device="cuda:0", stream=sa, **pa)
    gb = vp.VlasovRun(device="cuda:0", stream=sb, **pb)
    ga.init_conditions(fa)
    gb.init_conditions(fb)
    for k in range(13):
        ga.step(1)
        gb.step(1)
    ea, fa_ = ga.get_elements(), ga.reconstruct_f()
    eb, fb_ = gb.get_elements(), gb.reconstruct_f()
    ga.sync()
    gb.sync()
    assert np.array_equal(ea.cpu().numpy(), ref_a[0])
    assert np.array_equal(fa_.cpu().numpy(), ref_a[1])
    assert np.array_equal(eb.cpu().numpy(), ref_b[0])
    assert np.array_equal(fb_.cpu().numpy(), ref_b[1])
