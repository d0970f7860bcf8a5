"""E_map (neighbour mismatch of the predicted Lagrangian positions, end of
section 2.3.3) and the adaptive resampling it drives, against the oracle.

E_map is a maximum of per-site values computed with the same operations on
both sides, so for one element state it must agree exactly; an adaptive run
must follow the oracle's trajectory (to the rounding of the density sums,
tests/parity.py), remapping at the same checks."""
import numpy as np
import pytest

import workloads as W
from parity import RTOL, assert_elements_close, rel_linf

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def halos(n, seed=7, k=3):
    rng = np.random.default_rng(seed)
    box = (-1.0, 1.0, -1.0, 1.0)
    return W.finish(W.halo_sum(n, n, box, rng, k), box, 1.0)


def pair(vp, orc, p, f0, precision="fp64"):
    o = orc.Oracle(**p)
    o.init_conditions(f0)
    g = vp.VlasovRun(device="cuda:0", precision=precision, **p)
    g.init_conditions(f0)
    return o, g


@pytest.mark.parametrize("case", ["self", "anharmonic", "perturbed"])
def test_emap_matches_oracle(vp, orc, case):
    n, s = 128, 8
    p = dict(nx=n, sx=s, dt=2e-3, n_s=40)
    if case == "anharmonic":
        p.update(force_mode=1, ext=(0.1, -1.3, 2.1), dt=0.02)
    o, g = pair(vp, orc, p, halos(n))
    assert g.diagnostics()["emap"] == o.emap() == 0.0
    o.step(25)
    g.step(25)
    if case == "anharmonic":
        # no density sum enters an external force: the same trajectory
        assert np.array_equal(g.get_elements().cpu().numpy(),
                              o.get_elements())
    else:
        assert_elements_close(g.get_elements().cpu().numpy(), o)
    el = o.get_elements()
    if case == "perturbed":
        rng = np.random.default_rng(5)
        el[6:] += rng.uniform(-3.0, 3.0, el[6:].shape)
        el[2:6] += rng.uniform(-0.1, 0.1, el[2:6].shape)
        o.set_elements(el)
    g.set_elements(el)
    e_ref = o.emap()
    assert e_ref > 0.0
    assert g.diagnostics()["emap"] == e_ref
    g.sync()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adaptive_remap_follows_oracle(vp, orc, precision):
    """Self-gravitating halos, no fixed cadence, E_map checked every 4
    steps against a threshold that the run crosses: the FP64 engine keeps
    the oracle's elements and f (so it resamples at the same checks: a
    different decision would restart the elements at another step); mixed
    precision keeps f within 1e-5."""
    n, s = 128, 8
    p = dict(nx=n, sx=s, dt=4e-3, n_s=0)
    probe = orc.Oracle(**p)
    probe.init_conditions(halos(n))
    probe.step(8)
    thr = 0.5 * probe.emap()
    p.update(emap_max=thr, emap_every=4)
    o, g = pair(vp, orc, p, halos(n), precision)
    o.step(24)
    g.step(24)
    el_ref = o.get_elements()
    # at least one adaptive resampling happened: the elements restarted
    # from the lattice after t = 0
    free = orc.Oracle(**dict(p, emap_max=0.0, emap_every=0))
    free.init_conditions(halos(n))
    free.step(24)
    assert not np.array_equal(free.get_elements(), el_ref)
    if precision == "fp64":
        assert_elements_close(g.get_elements().cpu().numpy(), o)
        f_ref = o.reconstruct_f()
        assert rel_linf(g.reconstruct_f().cpu().numpy(), f_ref) <= RTOL
    else:
        f_ref = o.reconstruct_f()
        f = g.reconstruct_f().cpu().numpy().astype(np.float64)
        assert np.linalg.norm(f - f_ref) / np.linalg.norm(f_ref) <= 1e-5
    g.sync()


def test_server_rejects_adaptive_requests(vp):
    import torch
    n = 64
    f0 = torch.as_tensor(halos(n), device="cuda:0")
    out = torch.empty((n, n), dtype=torch.float64, device="cuda:0")
    srv = vp.Server(precision="fp64", max_active=2, pool_bytes=1 << 26)
    res, st = srv.run([dict(params=dict(nx=n, sx=4, dt=1e-3, n_s=10,
                                        precision="fp64", emap_max=0.1,
                                        emap_every=2),
                            f0=f0, out=out, nsteps=3, tag=1,
                            arrival_s=0.0)])
    assert res[0]["status"] == vp.EINVAL and st["completed"] == 1
    srv.close()
