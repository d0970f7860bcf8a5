"""vp_poisson_static (no run context, no workspace: the field's scratch in a
library-owned device array) against vp_poisson of a run context, through
the C ABI: bit for bit, on two calls in a row, the second with a smaller
grid, for both field paths (one workgroup up to 2048 columns, the chunked
launches above), isolated and periodic x, and at the maximum size."""
import math

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def vp():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1705_03750_amd as vp
    vp.lib()
    return vp


def context_poisson(vp, rho, kw):
    g = vp.VlasovRun(device="cuda:0", nx=len(rho), nv=16, **kw)
    out = [t.cpu().numpy() for t in g.poisson(rho)]
    g.sync()
    g.close()
    return out


def params_for(nx, bc):
    kw = dict(sx=8 if nx % 8 == 0 else 4, sv=8, dt=1e-3, G=0.7)
    if bc:
        kw.update(bc=1, x_min=0.0, x_max=4.0 * math.pi, G=-0.5)
    return kw


@pytest.mark.parametrize("bc,sizes", [(0, (4100, 1000)), (1, (4096, 1024)),
                                      (0, (16384, 2304))])
def test_static_poisson_equals_context_poisson(vp, bc, sizes):
    import torch
    rng = np.random.default_rng(sum(sizes) + bc)
    for nx in sizes:
        kw = params_for(nx, bc)
        rho = rng.uniform(0.0, 2.0, nx)
        print(f"[poisson_static] bc={bc} nx={nx}", flush=True)
        ref = context_poisson(vp, rho, kw)
        got = vp.poisson_static(torch.as_tensor(rho, device="cuda:0"),
                                nv=16, **kw)
        torch.cuda.synchronize()
        for name, x, y in zip(("a", "da", "d2a"), got, ref):
            assert np.array_equal(x.cpu().numpy(), y), (name, nx)


def test_static_poisson_rejects_oversize(vp):
    import torch
    nx = 16384 + 8
    rho = torch.zeros(nx, dtype=torch.float64, device="cuda:0")
    with pytest.raises(vp.VPError) as ei:
        vp.poisson_static(rho, nv=16, sx=8, sv=8, dt=1e-3)
    assert ei.value.code == vp.EINVAL
