"""Host-side checks of the HIP library that need no GPU: it loads, exports every symbol the
header declares, and rejects invalid configurations synchronously."""
import ctypes
import os
import re

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lbrbc.h")


def test_library_exports_every_declared_symbol():
    from paper_1107_4889_amd import lbrbc

    text = open(HEADER).read()
    declared = set(re.findall(r"^\s*(?:lb_status|void|const char\*)\s+(\w+)\s*\(", text, re.M))
    assert len(declared) >= 20
    lib = ctypes.CDLL(lbrbc.LIB_PATH)
    missing = [s for s in sorted(declared) if not hasattr(lib, s)]
    assert not missing, missing
    assert declared == set(lbrbc.SYMBOLS)


def _cfg(**kw):
    from paper_1107_4889_amd import lbrbc
    d = dict(nx=16, ny=16, nz=32, periodic=(0, 0, 1), tau0=0.8)
    d.update(kw)
    return lbrbc.make_config(d)


def test_footprint_and_validation_on_host():
    from paper_1107_4889_amd import lbrbc, synth

    solid = synth.tube(16, 16, 32, 6.0)
    b32 = lbrbc.lb_query_footprint(_cfg(storage="f32"), solid, 10)
    b64 = lbrbc.lb_query_footprint(_cfg(storage="f64"), solid, 10)
    b16 = lbrbc.lb_query_footprint(_cfg(storage="bf16"), solid, 10)
    N = 16 * 16 * 32
    assert b64 > b32 > b16 >= 2 * 19 * N * 2
    for ok in (2.0 ** 21, 2.0 ** 10, 2.0 ** 40):
        assert lbrbc.lb_query_footprint(_cfg(storage="f16", f16_scale=ok), solid, 10) > 0
    # FP16 scales below 2^10 let slow flows underflow silently; a scale must be a power of two
    for bad in (dict(tau0=0.5), dict(map_cap=13), dict(storage=7), dict(open_z=1),
                dict(nx=0), dict(xi=(0, 1, 1)), dict(storage="f16", f16_scale=3.0),
                dict(storage="f16", f16_scale=0.0), dict(storage="f16", f16_scale=2.0 ** 41),
                dict(storage="f16", f16_scale=2.0 ** 9), dict(storage="f16", f16_scale=1.0),
                dict(cand_cap=-1), dict(wall_u_hi=(float("nan"), 0, 0)),
                dict(periodic=(0, 0, 0), open_z=1, wall_u_lo=(1e-3, 0, 0))):
        with pytest.raises(lbrbc.LbError) as e:
            lbrbc.lb_query_footprint(_cfg(**bad), solid, 10)
        assert e.value.status == lbrbc.LB_EINVAL
    # a periodic axis shorter than a support tile is rejected when cells are present
    with pytest.raises(lbrbc.LbError):
        lbrbc.lb_query_footprint(_cfg(nz=12), synth.tube(16, 16, 12, 6.0), 3)
    assert lbrbc.lb_query_footprint(_cfg(nz=12), synth.tube(16, 16, 12, 6.0), 0) > 0


def test_null_arguments_are_rejected():
    from paper_1107_4889_amd import lbrbc
    L = lbrbc._lib
    assert L.lb_step(None, 1) == lbrbc.LB_EINVAL
    assert L.lb_sync(None) == lbrbc.LB_EINVAL
    assert L.rbc_couple(None) == lbrbc.LB_EINVAL
    assert L.lb_query_footprint(None, None, 0, None) == lbrbc.LB_EINVAL
    assert L.lb_set_stream(None, None) == lbrbc.LB_EINVAL
    arr = (lbrbc._P * 1)(None)
    ns = (ctypes.c_int * 1)(3)
    assert L.lb_batch_step(arr, ns, 1) == lbrbc.LB_EINVAL          # a NULL context
    assert L.lb_batch_step(None, ns, 1) == lbrbc.LB_EINVAL
    assert L.lb_batch_step(arr, ns, 0) == lbrbc.LB_OK              # nothing to do


def test_too_many_cells_for_coverage_entries():
    # entries are cell << shift | j in 32 bits: the shift for xi = (4, 4, 1.5) is 11, so at
    # most 2^20 cells fit
    from paper_1107_4889_amd import lbrbc, synth

    solid = synth.tube(16, 16, 32, 6.0)
    assert lbrbc.lb_query_footprint(_cfg(), solid, (1 << 20) - 1) > 0
    with pytest.raises(lbrbc.LbError) as e:
        lbrbc.lb_query_footprint(_cfg(), solid, 1 << 20)
    assert e.value.status == lbrbc.LB_EINVAL


def test_binding_fails_loudly_without_the_library(tmp_path):
    # the binding has no fallback: imported from a package folder without liblbrbc.so it
    # raises ImportError naming the missing library
    import shutil
    import subprocess
    import sys

    pkg = tmp_path / "nolib_pkg"
    pkg.mkdir()
    (pkg / "__init__.py").write_text("")
    src = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                       "paper_1107_4889_amd", "lbrbc.py")
    shutil.copy(src, pkg / "lbrbc.py")
    r = subprocess.run([sys.executable, "-c", "import nolib_pkg.lbrbc"], cwd=tmp_path,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode != 0
    assert "ImportError" in r.stderr and "liblbrbc.so is not built" in r.stderr


def test_planes_over_4_gib_are_rejected():
    # Per-node planes are addressed with 32-bit byte offsets: a 1024 x 1024 x 1025 FP32 lattice
    # (2^30 + 2^20 nodes, 4-byte u and sigma planes over 4 GiB) and a 1024 x 1024 x 513 FP64
    # one are rejected before any geometry is built; 1024 x 1024 x 1023 FP32 passes that check.
    from paper_1107_4889_amd import lbrbc

    for nz, storage in ((1025, "f32"), (1025, "bf16"), (513, "f64")):
        solid = np.zeros(1024 * 1024 * nz, dtype=np.uint8)     # never read: rejected first
        with pytest.raises(lbrbc.LbError) as e:
            lbrbc.lb_query_footprint(_cfg(nx=1024, ny=1024, nz=nz, storage=storage), solid, 0)
        assert e.value.status == lbrbc.LB_EINVAL
        assert "32-bit plane offsets" in str(e.value)
