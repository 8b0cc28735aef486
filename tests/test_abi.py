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
              "cutcell_build_transpose", "cutcell_transpose_workspace_bytes", "cutcell_backward_workspace_bytes",
              "cutcell_solve", "cutcell_solve_workspace_bytes", "cutcell_laplacian_count", "cutcell_laplacian_fill",
              "cutcell_apply_laplacian", "cutcell_laplacian_workspace_bytes", "cutcell_last_reused_faces", "cutcell_last_qr_faces",
              "cutcell_ritz", "cutcell_ritz_workspace_bytes", "cutcell_hessenberg_eigs", "cutcell_pack_count",
              "cutcell_pack_fill", "cutcell_apply_packed", "cutcell_pack_workspace_bytes", "cutcell_last_bin_faces"):
        assert n in names


def test_library_exports_every_declared_symbol(lib):
    for name in _declared():
        assert hasattr(lib, name), name
        assert name in _lib.SIGNATURES, f"binding lacks {name}"


def test_abi_version(lib):
    assert lib.cutcell_abi_version() == 12


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
    assert lib.cutcell_apply(ctypes.byref(sizes), 4, ctypes.byref(st), 8, 8, 8, None) == _lib.E_UNSUPPORTED
    # an empty batch (no volumes, no faces) needs no arrays at all
    assert lib.cutcell_apply(ctypes.byref(sizes), 3, None, None, None, None, None) == _lib.OK
    it = ctypes.c_int32(-1)
    assert lib.cutcell_solve(ctypes.byref(sizes), 3, None, None, None, None, None, 10, 10, 1e-8, None, 0,
                             ctypes.byref(it), None, None) == _lib.OK and it.value == 0
    full = _lib.Sizes(n_vol=10, n_eb=0, n_box=4, n_phi=14, n_face=20, nnz=100, max_rows=5, n_geom=1)
    assert lib.cutcell_apply(ctypes.byref(full), 3, ctypes.byref(st), None, None, None, None) == _lib.E_INVALID_ARG
    assert lib.cutcell_apply_laplacian(ctypes.byref(full), 3, None, None, None, None) == _lib.E_INVALID_ARG


def _fake_stencils():
    arr = _lib.StencilArrays()
    for name in ("row_ptr", "col", "val", "status", "vol_face", "vol_scale", "phi_off", "vol_off", "face_off"):
        setattr(arr, name, 8)
    return arr


@pytest.mark.parametrize("restart,max_iters,rtol,code", [
    (0, 10, 1e-8, _lib.E_INVALID_ARG),
    (1025, 10, 1e-8, _lib.E_INVALID_ARG),
    (10, -1, 1e-8, _lib.E_INVALID_ARG),
    (10, 10, -1.0, _lib.E_INVALID_ARG),
    (10, 10, float("nan"), _lib.E_INVALID_ARG),
])
def test_solve_rejects_bad_arguments_on_the_host(lib, restart, max_iters, rtol, code):
    """Argument checks come before any device work, so these run without a GPU."""
    sizes = _lib.Sizes(n_vol=10, n_eb=0, n_box=4, n_phi=14, n_face=20, nnz=100, max_rows=5, n_geom=1)
    arr = _fake_stencils()
    it = ctypes.c_int32(-1)
    rc = lib.cutcell_solve(ctypes.byref(sizes), 2, ctypes.byref(arr), None, 8, 8, 8, restart, max_iters, rtol, 8,
                           1 << 20, ctypes.byref(it), None, None)
    assert rc == code
    assert lib.cutcell_last_error()


def test_solve_workspace_size(lib):
    sizes = _lib.Sizes(n_vol=1000, n_eb=10, n_box=40, n_phi=1050, n_face=3000, nnz=10**5, max_rows=30, n_geom=1)
    assert lib.cutcell_solve_workspace_bytes(ctypes.byref(sizes), 0) == 0
    assert lib.cutcell_solve_workspace_bytes(ctypes.byref(sizes), 1025) == 0
    b10 = lib.cutcell_solve_workspace_bytes(ctypes.byref(sizes), 10)
    b20 = lib.cutcell_solve_workspace_bytes(ctypes.byref(sizes), 20)
    assert b10 >= 8 * (11 * 1000 + 2 * 1050 + 3000)
    assert b20 - b10 >= 8 * 10 * 1000


def test_bad_boundary_condition_rejected(lib):
    o = _opts()
    o.eb_bc = 2
    g = _lib.Geom()
    g.vol_mom = 8
    for d in range(3):
        g.face_mom[d] = 8
    sizes = _lib.Sizes()
    rc = lib.cutcell_query(ctypes.byref(g), 1, ctypes.byref(o), None, 0, ctypes.byref(sizes), None)
    assert rc == _lib.E_INVALID_ARG
    assert b"eb_bc" in lib.cutcell_last_error()


def test_stencil_adjoint_rejects_neumann_on_the_host(lib):
    """The adjoint supports Dirichlet EB conditions only; the check precedes device work."""
    o = _opts()
    o.eb_bc = _lib.BC_NEUMANN
    g = _lib.Geom()
    g.vol_mom = 8
    for d in range(3):
        g.face_mom[d] = 8
    sizes = _lib.Sizes(n_vol=10, n_eb=0, n_box=4, n_phi=14, n_face=20, nnz=100, max_rows=5, n_geom=1)
    arr = _fake_stencils()
    tr = _lib.TransposeArrays()
    tr.col_ptr, tr.nz, tr.nz_face = 8, 8, 8
    gr = _lib.GeomGrad()
    gr.vol_mom = 8
    for d in range(3):
        gr.face_mom[d] = 8
    rc = lib.cutcell_stencils_backward(ctypes.byref(g), 1, ctypes.byref(o), ctypes.byref(sizes), ctypes.byref(arr),
                                       ctypes.byref(tr), 8, None, ctypes.byref(gr), None, 8, 1 << 20, None)
    assert rc == _lib.E_UNSUPPORTED
    assert b"Dirichlet" in lib.cutcell_last_error()


def test_one_fourth_order_64_cubed_geometry_fits_the_static_scratch(lib):
    """The no-allocation build's scratch holds the workspace of one 64^3 order-4 geometry
    (the header's promise), and a batch of four 48^3 ones exceeds it."""
    from paper_1411_4283_amd.api import make_opts

    o = make_opts(3, (64, 64, 64), 1 / 64, 4, 3)
    assert 0 < lib.cutcell_workspace_bytes(ctypes.byref(o), 1) <= _lib.STATIC_SCRATCH_BYTES
    o48 = make_opts(3, (48, 48, 48), 1 / 48, 4, 3)
    assert lib.cutcell_workspace_bytes(ctypes.byref(o48), 4) > _lib.STATIC_SCRATCH_BYTES
