"""cutcell_build_stencils_noalloc: the stencil build with the library's static scratch in
place of a caller workspace, for callers that cannot allocate device memory.  Called
through the C ABI twice in a row, the second time on a smaller input, it must give
bit for bit the outputs of cutcell_build_stencils on the same inputs (the same kernels,
only the scratch differs); inputs too large for the scratch are refused."""

import ctypes

import numpy as np
import pytest

import cutgeom as cg

torch = pytest.importorskip("torch")
import paper_1411_4283_amd as cc  # noqa: E402
from paper_1411_4283_amd import _lib  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _outputs(st):
    s = st.sizes
    return [st.row_ptr, st.col[: s.nnz], st.val[: s.nnz].view(torch.int64), st.status[: s.n_face],
            st.vol_face[: s.n_vol * (2 * st.dim + 1)], st.vol_scale[: s.n_vol].view(torch.int64), st.phi_off,
            st.vol_off, st.face_off]


def _noalloc_build(b):
    out = b.allocate()
    arr = out.struct()
    rc = _lib.load().cutcell_build_stencils_noalloc(b.garr, len(b.geoms), ctypes.byref(b.opts),
                                                    ctypes.byref(b.sizes), ctypes.byref(arr),
                                                    ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    out.code = _lib.check(rc, "cutcell_build_stencils_noalloc")
    torch.cuda.synchronize()
    return out


@pytest.mark.parametrize("qr", [False, True])
def test_noalloc_build_matches_the_workspace_build_twice(qr):
    fac = "qr" if qr else "auto"
    # the 64^3 fourth-order workload (the largest the scratch promises to hold), then smaller
    cases = [(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 64, 4, 3), (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 20, 4, 3),
             (cg.ball_outside((0.5, 0.5), 0.25), 24, 2, 2)]
    for shape, n, Q, R in cases:          # the second call has the smaller input
        g = cg.make_geometry(shape, n, Q)
        dg = cc.DeviceGeometry.from_host(g, DEV)
        b = cc.Builder(dg, R, factorization=fac)
        ref = b.build()
        torch.cuda.synchronize()
        got = _noalloc_build(b)
        assert got.code == ref.code
        for x, y in zip(_outputs(got), _outputs(ref)):
            assert torch.equal(x, y)
        _say(f"noalloc {g.D}D n={n} Q={Q} ({fac}): {ref.sizes.n_face} faces, identical")


def test_noalloc_refuses_inputs_beyond_the_scratch():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 12, 4)
    dgs = [cc.DeviceGeometry.from_host(g, DEV)]
    b = cc.Builder(dgs, 3)
    b.query()
    lib = _lib.load()
    need = lib.cutcell_workspace_bytes(ctypes.byref(b.opts), 1)
    assert 0 < need <= _lib.STATIC_SCRATCH_BYTES
    # a batch whose workspace exceeds the scratch is refused before anything runs
    big = [cc.DeviceGeometry.from_host(cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 48, 4), DEV)] * 4
    bb = cc.Builder(big, 3)
    assert lib.cutcell_workspace_bytes(ctypes.byref(bb.opts), 4) > _lib.STATIC_SCRATCH_BYTES
    bb.query()
    with pytest.raises(_lib.CutcellError) as e:
        _noalloc_build(bb)
    assert e.value.code == _lib.E_WORKSPACE
