"""Degenerate inputs through the C ABI: a box with no embedded boundary at all (every cell
full, only box faces as boundary rows), and a box with no fluid (no volumes, no faces),
through the build, the apply, the volume matrix, template reuse and the solve."""

import numpy as np
import pytest

import cutgeom as cg
import oracle

torch = pytest.importorskip("torch")
import paper_1411_4283_amd as cc  # noqa: E402
from test_gpu_parity import _check_apply, _host  # noqa: E402
from test_gpu_solve import _exact_phi_and_rhs, _t  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


@pytest.mark.parametrize("D,Q,R,n", [(2, 4, 3, 12), (3, 2, 2, 8)])
def test_all_fluid_box(D, Q, R, n):
    nrm = [0.0] * D
    nrm[-1] = 1.0
    g = cg.make_geometry(cg.halfspace(nrm, -1.0), n, Q)      # fluid everywhere
    assert len(g.eb_cell) == 0 and np.all(g.kappa == 1.0)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    st = cc.Builder(dg, R).build()
    en, rp, col, val, status = oracle.build(g, R)
    rp_g, col_g, val_g, st_g = _host(st)
    assert st.sizes.n_eb == 0 and st.sizes.n_vol == n**D
    assert np.array_equal(rp_g, rp) and np.array_equal(col_g, col) and np.array_equal(st_g, status)
    ok = status == oracle.STATUS_OK
    for f in np.flatnonzero(ok):
        a, e = rp[f], rp[f + 1]
        assert np.abs(val_g[a:e] - val[a:e]).max() <= 1e-11 * np.abs(val[a:e]).max()
    _check_apply(g, en, st, rp_g, col_g, val_g, np.random.default_rng(3).standard_normal(en.n_phi))
    # reuse and the volume matrix agree with the plain build; the solve is exact for
    # polynomials of degree <= Q
    reuse = cc.Builder(dg, R, reuse_templates=True).build()
    assert torch.equal(reuse.val, st.val) and reuse.reused > 0
    lap = cc.build_laplacian(st)
    phi, rhs = _exact_phi_and_rhs(g, en, cg.random_polynomial(D, Q, np.random.default_rng(4), scale=0.5))
    res = cc.solve(st, _t(phi), _t(rhs), rtol=1e-13, lap=lap)
    assert res.converged
    assert np.abs(res.x.cpu().numpy() - phi[: en.n_vol]).max() <= 1e-9 * np.abs(phi).max()


def test_no_fluid():
    g = cg.make_geometry(cg.halfspace([0.0, 1.0], 2.0), 16, 4)   # fluid nowhere in the box
    assert np.all(g.kappa == 0.0)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    st = cc.Builder(dg, 3).build()
    s = st.sizes
    assert (s.n_vol, s.n_face, s.nnz, s.n_phi) == (0, 0, 0, 0)
    L, flux = cc.apply(st, torch.zeros(0, dtype=torch.float64, device=DEV))
    assert L.numel() == 0 and flux.numel() == 0
    lap = cc.build_laplacian(st)
    assert lap.nnz == 0 and int(lap.row_ptr[0]) == 0
    res = cc.solve(st, torch.zeros(1, dtype=torch.float64, device=DEV)[:0], torch.zeros(0, dtype=torch.float64,
                                                                                         device=DEV))
    assert res.converged and res.iters == 0
