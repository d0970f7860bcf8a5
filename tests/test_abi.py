"""The C-ABI library loads, exports every entry point include/vp.h declares,
and validates parameters on the host (no device work)."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    src = open(os.path.join(ROOT, "include", "vp.h")).read()
    return sorted(set(re.findall(r"\b(vp_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def vp():
    import paper_1705_03750_amd as vp
    if not os.path.exists(vp.LIB_PATH):
        from paper_1705_03750_amd import build
        build.build()
    return vp


def test_exports_every_declared_symbol(vp):
    L = C.CDLL(vp.LIB_PATH)
    names = _declared()
    assert "vp_step" in names and "vp_reconstruct_f" in names
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    assert set(vp.EXPORTS) == set(names)


def test_footprint_and_validation(vp):
    n_fp64 = vp.footprint(nx=256, sx=4, dt=1e-3)
    n_mixed = vp.footprint(nx=256, sx=4, dt=1e-3, precision="mixed")
    assert n_fp64 > n_mixed > 0
    big = vp.footprint(nx=2048, sx=8, dt=5e-4)
    assert 3 * 2048 * 2048 * 8 < big < 8 * 2048 * 2048 * 8
    for bad in (dict(nx=250, sx=4, dt=1e-3),      # nx % sx
                dict(nx=4, sx=1, dt=1e-3),        # too small
                dict(nx=30, sx=3, dt=1e-3),       # nx % 4
                dict(nx=64, sx=4, dt=0.0),        # dt <= 0
                dict(nx=64, sx=4, dt=1e-3, x_min=1.0, x_max=1.0),
                dict(nx=64, sx=4, dt=1e-3, n_s=-1),
                dict(nx=64, sx=4, dt=1e-3, precision=7),
                dict(nx=64, sx=4, dt=1e-3, c_dyn=-0.5),
                dict(nx=64, sx=4, dt=1e-3, c_dyn=float("inf")),
                # the variable step needs the self-consistent density
                dict(nx=64, sx=4, dt=1e-3, c_dyn=0.1, force_mode=1),
                dict(nx=36, sx=4, dt=1e-3, bc=1),   # periodic: nx % 8
                dict(nx=64, sx=4, dt=1e-3, bc=1, force_mode=1),
                dict(nx=64, sx=4, dt=1e-3, bc=2)):
        with pytest.raises(vp.VPError) as ei:
            vp.footprint(**bad)
        assert ei.value.code == vp.EINVAL


def test_create_rejects_small_or_null_workspace(vp):
    p = vp.make_params(nx=64, sx=4, dt=1e-3)
    n = C.c_size_t(0)
    assert vp.lib().vp_footprint(C.byref(p), C.byref(n)) == 0
    h = C.c_void_p()
    # null workspace and short workspace are refused before any device work
    assert vp.lib().vp_create(C.byref(p), None, n.value, None,
                              C.byref(h)) == vp.EINVAL
    assert vp.lib().vp_create(C.byref(p), C.c_void_p(256), n.value - 1, None,
                              C.byref(h)) == vp.ENOMEM
    assert b"vp_footprint" in vp.lib().vp_last_error(None)


def test_vp4_exports_and_validation():
    """The 4D library loads (no GPU needed), exports every symbol its
    header declares, and validates parameters."""
    import ctypes as C
    import re
    import paper_1705_03750_amd.vp4 as v4
    L = v4.lib()
    hdr = open(os.path.join(ROOT, "include", "vp4.h")).read()
    declared = set(re.findall(r"\b(vp4_[a-z_]+)\s*\(", hdr))
    assert declared == set(v4.EXPORTS)
    for name in declared:
        getattr(L, name)
    n = C.c_size_t(0)
    ok = v4.make_params(ns=16, nv=8, L=1.0, vmax=1.0, ss=4, sv=4)
    assert L.vp4_footprint(C.byref(ok), C.byref(n)) == 0 and n.value > 0
    for bad in (dict(ns=18, nv=8, L=1.0, vmax=1.0, ss=2, sv=4),
                dict(ns=16, nv=6, L=1.0, vmax=1.0, ss=4, sv=2),
                dict(ns=16, nv=8, L=0.0, vmax=1.0, ss=4, sv=4),
                dict(ns=16, nv=8, L=1.0, vmax=1.0, ss=4, sv=4, precision=3)):
        p = v4.make_params(**bad)
        assert L.vp4_footprint(C.byref(p), C.byref(n)) == v4.VP4Error(
            -1, "").code


def test_bench_refuses_more_than_one_gpu():
    """bench.py runs on one GPU: --gpus 2 exits with status 2 and a message,
    before touching a device."""
    import subprocess
    import sys
    import os
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    r = subprocess.run([sys.executable, os.path.join(root, "bench.py"),
                        "--gpus", "2"], capture_output=True, text=True,
                       timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_traffic_record_follows_the_kernel_code(tmp_path, monkeypatch):
    """The measured-traffic record is tied to the engine's code: the hash
    bench.py checks ignores comments and blank lines but changes with any
    code token."""
    import shutil
    import sys
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    sys.path.insert(0, root)
    import bench
    rel = ("paper_1705_03750_amd/csrc/vp_kernels.hpp",
           "paper_1705_03750_amd/csrc/vp_engine.hip")
    for f in rel:
        os.makedirs(tmp_path / os.path.dirname(f), exist_ok=True)
        shutil.copy(os.path.join(root, f), tmp_path / f)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    h0 = bench.kernel_source_hash()
    eng = tmp_path / rel[1]
    text = eng.read_text()
    eng.write_text("// a new comment\n\n/* and a block\n comment */\n" +
                   text.replace("\n", "  // trailing\n", 3))
    assert bench.kernel_source_hash() == h0
    eng.write_text(text.replace("GRID_TILE = 8192", "GRID_TILE = 4096"))
    assert bench.kernel_source_hash() != h0


def test_poisson_static_validates_on_the_host(vp):
    """vp_poisson_static's argument checks come before any device work:
    null pointers and nx above VP_POISSON_STATIC_MAX_NX give EINVAL with a
    message in vp_last_error(NULL)."""
    L = vp.lib()
    p = vp.make_params(nx=64, sx=8, dt=1e-3)
    assert L.vp_poisson_static(C.byref(p), None, None, None, None,
                               None) == vp.EINVAL
    big = vp.make_params(nx=16384 + 8, sx=8, dt=1e-3)
    fake = C.c_void_p(256)  # never dereferenced: rejected first
    assert L.vp_poisson_static(C.byref(big), fake, fake, fake, fake,
                               None) == vp.EINVAL
    assert b"VP_POISSON_STATIC_MAX_NX" in L.vp_last_error(None)
