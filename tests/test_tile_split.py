"""Host logic of the reconstruction's tile split (not a GPU test).

The engine splits a tile index t < nbx * ngy into (bx, gy) with the
multiplier m = ceil(2^40 / nbx): gy = (t m) >> 40.  It is exact for every t
when nbx^2 ngy < 2^40, since the rounding excess of m adds less than
t / 2^40 < 1 / nbx to t / nbx.  These tests check that claim by brute force
on the block geometry the engine derives from (nx, nv, sv), including the
largest grids the parameters allow, and that those grids meet the bound.
"""
import numpy as np
import pytest


def geometry(nx, nv, sv):
    # the engine's block counts: nbx = (nx - 1) / 8 + 2 block columns,
    # ngy = (nv - 1 - ov) / 64 + obv + 1 row groups, ov = (sv / 2) % 8
    ov = (sv // 2) % 8
    obv = 1 if ov > 0 else 0
    nbx = ((nx - 1) >> 3) + 2
    ngy = ((nv - 1 - ov) >> 6) + obv + 1
    return nbx, ngy


def split_exact(nbx, ngy):
    m = ((1 << 40) + nbx - 1) // nbx
    t = np.arange(nbx * ngy, dtype=np.uint64)
    gy = (t * np.uint64(m)) >> np.uint64(40)
    return bool(np.array_equal(gy, t // np.uint64(nbx)))


@pytest.mark.parametrize("nx,nv,sv", [
    (8, 8, 1), (2048, 2048, 8), (1020, 1004, 4), (8192, 8192, 8),
    (16384, 16384, 16), (131072, 8, 1), (8, 131072, 2), (131072, 131072, 1),
    (131072, 131072, 16), (100000, 99996, 3)])
def test_multiplier_split_is_exact(nx, nv, sv):
    nbx, ngy = geometry(nx, nv, sv)
    assert nbx * nbx * ngy < (1 << 40)   # the engine's condition holds
    assert split_exact(nbx, ngy)


def test_bound_is_needed():
    # a geometry beyond the bound where the multiplier split fails, so the
    # condition is not vacuous
    nbx, ngy = 60000, 1 << 12
    assert nbx * nbx * ngy >= (1 << 40)
    m = ((1 << 40) + nbx - 1) // nbx
    t = nbx * ngy - 1
    assert ((t * m) >> 40) != t // nbx
