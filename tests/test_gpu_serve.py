"""Continuous-batching server: every request's result is bitwise the same
alone, in a mix, and as a standalone run; admission waits for memory; an
FP64 request matches the CPU oracle."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def make_mix(torch, precision, count=6, seed=90, n_fixed=None, s_fixed=None):
    rng = np.random.default_rng(seed)
    box = (-1.0, 1.0, -1.0, 1.0)
    reqs = []
    t = 0.0
    for i in range(count):
        n = int(rng.choice([64, 96, 128]))
        s = int(rng.choice([4, 8]))
        n = n_fixed or n
        s = s_fixed or s
        nsteps = int(rng.integers(20, 61))
        n_s = int(rng.choice([7, 10, 25]))
        f0 = W.finish(W.halo_sum(n, n, box, rng, int(rng.integers(1, 4))),
                      box, 1.0)
        fdt = torch.float32 if precision == "mixed" else torch.float64
        reqs.append(dict(
            params=dict(nx=n, sx=s, dt=2e-3, n_s=n_s, precision=precision),
            f0=torch.as_tensor(f0, device="cuda:0"),
            out=torch.full((n, n), float("nan"), dtype=fdt, device="cuda:0"),
            nsteps=nsteps, tag=100 + i, arrival_s=t))
        t += float(rng.uniform(0.0, 0.004))
    return reqs


def standalone(vp, r):
    p = dict(r["params"])
    prec = p.pop("precision")
    run = vp.VlasovRun(device="cuda:0", precision=prec, **p)
    run.init_conditions(r["f0"])
    run.step(r["nsteps"])
    f = run.reconstruct_f()
    run.sync()
    return f.cpu().numpy()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_mix_equals_alone_equals_standalone(vp, precision):
    import torch
    reqs = make_mix(torch, precision)
    srv = vp.Server(precision=precision, max_active=8, pool_bytes=1 << 28)
    res, st = srv.run(reqs)
    torch.cuda.synchronize()
    assert st["completed"] == len(reqs) and st["ticks"] > 0
    assert st["max_active"] >= 2           # runs overlapped on the device
    for r, x in zip(reqs, res):
        assert x["status"] == 0 and x["done_s"] >= x["admit_s"] >= 0
        got = r["out"].cpu().numpy()
        assert np.isfinite(got).all()
        ref = standalone(vp, r)
        assert np.array_equal(got, ref), r["tag"]
    # the first request served alone
    r0 = dict(reqs[0])
    r0["out"] = torch.full_like(reqs[0]["out"], float("nan"))
    r0["arrival_s"] = 0.0
    srv.run([r0])
    torch.cuda.synchronize()
    assert np.array_equal(r0["out"].cpu().numpy(), reqs[0]["out"].cpu().numpy())
    srv.close()


def test_admission_waits_for_memory(vp):
    import torch
    # identical footprints, so the pool holds exactly two runs at a time
    reqs = make_mix(torch, "mixed", count=6, seed=91, n_fixed=96, s_fixed=4)
    for r in reqs:
        r["arrival_s"] = 0.0
    need = max(vp.footprint(**r["params"]) for r in reqs)
    import ctypes as C
    hdr = C.c_size_t(0)
    vp.lib().vp_server_footprint(vp.MIXED, C.byref(hdr))
    pool = hdr.value + 2 * (need + 4096)
    srv = vp.Server(precision="mixed", max_active=8, pool_bytes=pool)
    res, st = srv.run(reqs)
    torch.cuda.synchronize()
    assert st["completed"] == 6 and st["max_active"] <= 2
    assert any(x["admit_s"] > 0.0 for x in res)
    for r in reqs:
        assert np.array_equal(r["out"].cpu().numpy(), standalone(vp, r))
    srv.close()


def test_fp64_request_matches_oracle(vp, orc):
    import torch
    reqs = make_mix(torch, "fp64", count=3, seed=92)
    srv = vp.Server(precision="fp64", max_active=4, pool_bytes=1 << 27)
    srv.run(reqs)
    torch.cuda.synchronize()
    r = reqs[1]
    p = dict(r["params"])
    p.pop("precision")
    o = orc.Oracle(**p)
    o.init_conditions(r["f0"].cpu().numpy())
    o.step(r["nsteps"])
    ref = o.reconstruct_f()
    got = r["out"].cpu().numpy()
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
    srv.close()


def test_rejects_wrong_precision(vp):
    import torch
    reqs = make_mix(torch, "fp64", count=1, seed=93)
    srv = vp.Server(precision="mixed", max_active=2, pool_bytes=1 << 26)
    res, st = srv.run(reqs)
    assert res[0]["status"] == vp.EINVAL and st["completed"] == 1
    srv.close()


@pytest.mark.parametrize("precision", ["mixed", "fp64"])
def test_large_requests_equal_standalone(vp, orc, precision):
    """The upper end of the serving mix: 1024^2 and 2048^2 grids with
    element strides 4 and 8, run together through two resamplings each.
    Every request is bit for bit its standalone run (the batched kernels at
    these sizes); in FP64 one request also matches the oracle on a seeded
    sample of sites."""
    import torch
    rng = np.random.default_rng(95)
    box = (-1.0, 1.0, -1.0, 1.0)
    fdt = torch.float32 if precision == "mixed" else torch.float64
    reqs = []
    for i, (n, s) in enumerate([(1024, 4), (1024, 8), (2048, 4), (2048, 8)]):
        f0 = W.finish(W.halo_sum(n, n, box, rng, 3), box, 1.0)
        reqs.append(dict(
            params=dict(nx=n, sx=s, dt=5e-4, n_s=25, precision=precision),
            f0=torch.as_tensor(f0, device="cuda:0"),
            out=torch.full((n, n), float("nan"), dtype=fdt, device="cuda:0"),
            nsteps=60, tag=200 + i, arrival_s=0.002 * i))
    print(f"[serve large] {precision}", flush=True)
    srv = vp.Server(precision=precision, max_active=4, pool_bytes=1 << 30)
    res, st = srv.run(reqs)
    torch.cuda.synchronize()
    assert st["completed"] == len(reqs) and st["max_active"] >= 2
    for r, x in zip(reqs, res):
        assert x["status"] == 0
        got = r["out"].cpu().numpy()
        assert np.isfinite(got).all()
        assert np.array_equal(got, standalone(vp, r)), r["tag"]
    srv.close()
    if precision != "fp64":
        return
    r = reqs[1]
    n = r["params"]["nx"]
    p = dict(r["params"])
    p.pop("precision")
    o = orc.Oracle(**p)
    o.init_conditions(r["f0"].cpu().numpy())
    o.step(r["nsteps"])
    srng = np.random.default_rng(7)
    j, i = srng.integers(0, n, 4096), srng.integers(0, n, 4096)
    ref = o.reconstruct_sites(j.astype(np.int64) * n + i)
    got = r["out"].cpu().numpy()[j, i]
    assert np.abs(got - ref).max() <= 1e-12 * np.abs(ref).max()
