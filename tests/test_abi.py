"""The C ABI library loads, exports every symbol its header declares, and validates its
arguments on the host (no GPU needed: these calls return before any HIP call)."""

import ctypes
import os
import re

import pytest

from paper_1411_4283_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "cutcell.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(cutcell_[a-z_]+)\s*\(", src)))


@pytest.fixture(scope="module")
def lib():
    return _lib.load()


def test_header_declares_the_entry_points():
    names = _declared()
    for n in ("cutcell_query", "cutcell_build_stencils", "cutcell_apply", "cutcell_workspace_bytes",
              "cutcell_last_error", "cutcell_abi_version", "cutcell_stencils_backward", "cutcell_apply_adjoint",
              "cutcell_build_transpose", "cutcell_transpose_workspace_bytes", "cutcell_backward_workspace_bytes"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_abi_version(lib):
    assert lib.cutcell_abi_version() == 3


def _opts(**kw):
    base = dict(dim=3, n=(16, 16, 16), h=1 / 16, order=4, path_radius=3)
    base.update(kw)
    from paper_1411_4283_amd.api import make_opts

    return make_opts(base["dim"], base["n"], base["h"], base["order"], base["path_radius"])


def test_workspace_size_is_host_computed(lib):
    o = _opts()
    b1 = lib.cutcell_workspace_bytes(ctypes.byref(o), 1)
    b2 = lib.cutcell_workspace_bytes(ctypes.byref(o), 2)
    assert b1 > 16**3 * 4 and b2 > b1
    bad = _opts(dim=4)
    assert lib.cutcell_workspace_bytes(ctypes.byref(bad), 1) == 0


@pytest.mark.parametrize("kw,code", [
    (dict(order=3), _lib.E_UNSUPPORTED),
    (dict(dim=1), _lib.E_UNSUPPORTED),
    (dict(path_radius=0), _lib.E_UNSUPPORTED),
    (dict(path_radius=5), _lib.E_UNSUPPORTED),
    (dict(h=0.0), _lib.E_INVALID_ARG),
    (dict(n=(0, 16, 16)), _lib.E_INVALID_ARG),
])
def test_query_rejects_bad_options(lib, kw, code):
    o = _opts(**kw)
    g = _lib.Geom()
    g.vol_mom = 8
    for d in range(3):
        g.face_mom[d] = 8
    sizes = _lib.Sizes()
    rc = lib.cutcell_query(ctypes.byref(g), 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None)
    assert rc == code
    assert lib.cutcell_last_error()


def test_query_rejects_null_pointers_and_small_workspace(lib):
    o = _opts()
    g = _lib.Geom()
    sizes = _lib.Sizes()
    assert lib.cutcell_query(ctypes.byref(g), 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None) == _lib.E_INVALID_ARG
    g.vol_mom = 8
    for d in range(3):
        g.face_mom[d] = 8
    g.n_eb = 3            # EB count without EB arrays
    assert lib.cutcell_query(ctypes.byref(g), 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None) == _lib.E_INVALID_ARG
    g.n_eb = 0
    rc = lib.cutcell_query(ctypes.byref(g), 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None)
    assert rc == _lib.E_WORKSPACE
    assert b"workspace" in lib.cutcell_last_error()
    assert lib.cutcell_query(None, 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None) == _lib.E_INVALID_ARG
    assert lib.cutcell_query(ctypes.byref(g), 0, ctypes.byref(o), None, 0, ctypes.byref(sizes), None) == _lib.E_INVALID_ARG


def test_build_and_apply_reject_null_outputs(lib):
    o = _opts()
    g = _lib.Geom()
    sizes = _lib.Sizes()
    st = _lib.StencilArrays()
    assert lib.cutcell_build_stencils(ctypes.byref(g), 1, ctypes.byref(o), ctypes.byref(sizes), ctypes.byref(st),
                                      None, 0, None) == _lib.E_INVALID_ARG
    assert lib.cutcell_apply(ctypes.byref(sizes), 3, ctypes.byref(st), None, None, None, None) == _lib.E_INVALID_ARG
    assert lib.cutcell_apply(ctypes.byref(sizes), 4, ctypes.byref(st), 8, 8, 8, None) == _lib.E_UNSUPPORTED
