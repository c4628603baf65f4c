"""CPU-side checks of the HIP library: it builds, loads, exports every entry
point declared in include/pbm.h, the Python binding covers them, and the
host-side validation rejects bad input before touching a device."""
import ctypes
import os
import re
import subprocess

import numpy as np
import pytest

import inputs

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pbm.h")


@pytest.fixture(scope="module")
def pbm():
    import paper_2108_10481_amd as p
    if not os.path.exists(p.LIB_PATH):
        from paper_2108_10481_amd import build
        build.build()
    p.load()
    return p


def declared_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pb_[a-z_]+)\s*\(", text)))


def test_header_declares_entry_points():
    names = declared_functions()
    assert "pb_solve" in names and "pb_mesh_apply" in names and len(names) >= 15


def test_library_exports_every_declared_symbol(pbm):
    lib = ctypes.CDLL(pbm.LIB_PATH)
    for name in declared_functions():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", pbm.LIB_PATH], capture_output=True, text=True).stdout
    exported = set(re.findall(r" T (pb_\w+)", out))
    assert set(declared_functions()) <= exported
    assert set(pbm.EXPORTS) == set(declared_functions())


def test_library_is_gfx950_code_object(pbm):
    out = subprocess.run(["strings", pbm.LIB_PATH], capture_output=True, text=True).stdout
    assert "gfx950" in out


def test_default_options_match_paper(pbm):
    o = pbm.pb_default_options()
    assert (o.eps_in, o.eps_out, o.kappa, o.tol) == (4.0, 80.0, 0.125, 1e-5)
    assert o.formulation == pbm.PB_DIRECT_INT and o.preconditioner == pbm.PB_BLOCK_DIAG
    assert o.singular_order == 4 and o.max_iter == 1000


def _create_status(pbm, xyz, tri, **kw):
    try:
        h = pbm.MeshHandle(xyz, tri, pbm.pb_default_options(**kw))
        h.close()
        return 0
    except pbm.PbError as e:
        return e.code


def test_host_validation_rejects_bad_meshes(pbm):
    m = inputs.icosphere(2, 1.0)
    # open mesh
    assert _create_status(pbm, m.xyz, m.tri[:-1]) == pbm.PB_E_MESH
    # inverted orientation
    assert _create_status(pbm, m.xyz, m.tri[:, ::-1].copy()) == pbm.PB_E_MESH
    # one flipped triangle: inconsistent orientation
    t = m.tri.copy()
    t[3] = t[3][::-1]
    assert _create_status(pbm, m.xyz, t) == pbm.PB_E_MESH
    # vertex id out of range
    t = m.tri.copy()
    t[0, 0] = 10 ** 6
    assert _create_status(pbm, m.xyz, t) == pbm.PB_E_MESH
    # degenerate triangle (collapsed vertex)
    x = m.xyz.copy()
    x[m.tri[0, 1]] = x[m.tri[0, 0]]
    assert _create_status(pbm, x, m.tri) == pbm.PB_E_MESH
    # non-finite coordinates and bad options
    x = m.xyz.copy()
    x[0, 0] = np.nan
    assert _create_status(pbm, x, m.tri) == pbm.PB_E_INVALID_ARG
    assert _create_status(pbm, m.xyz, m.tri, eps_in=-1.0) == pbm.PB_E_INVALID_ARG
    assert _create_status(pbm, m.xyz, m.tri, formulation=7) == pbm.PB_E_INVALID_ARG
    assert _create_status(pbm, m.xyz, m.tri, singular_order=0) == pbm.PB_E_INVALID_ARG


def test_valid_mesh_without_gpu_fails_loudly(pbm):
    if pbm.pb_device_count() > 0:
        pytest.skip("a GPU is present")
    m = inputs.icosphere(2, 1.0)
    assert _create_status(pbm, m.xyz, m.tri) == pbm.PB_E_DEVICE
    assert "device" in pbm.pb_last_error().lower()
