"""GPU parity of the adjoints (cutcell_apply_adjoint, cutcell_stencils_backward and the
autograd wrappers) against the oracle's adjoints, through the C ABI.

Bars (derived in the design notes; written in each test):
  * apply adjoint: per entry |d| <= 1e-12 * (sum of the magnitudes of the terms);
  * stencil gradients: per input array, max|g_gpu - g_orc| <= 1e-9 * max|g_orc|.  Each face
    contributes a bilinear form in (y, w, r, z), each of which both sides get from a
    refined or backward-stable solve with relative error <= ~cond(W A~) * eps; the faces'
    condition numbers stay below 1e6 here, so per-face errors are <= ~1e-10 relative and
    the sums over rows and faces add no cancellation beyond the largest term.
Faces outside the compared subset get val_bar = 0 (their gradient is then zero on both
sides), which keeps the oracle's per-face autograd within seconds.
"""

import numpy as np
import pytest

import cutgeom as cg
import oracle

torch = pytest.importorskip("torch")
import paper_1411_4283_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"
GRAD_TOL = 1e-9


def _say(msg):
    print(f"[gpu-adjoint] {msg}", flush=True)


CASES = {
    "circle16_q2": (cg.ball_outside((0.5, 0.5), 0.25), 16, 2, 2, None),
    "circle16_q4": (cg.ball_outside((0.5, 0.5), 0.25), 16, 4, 3, 160),
    "sphere10_q4": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 10, 4, 3, 90),
    "sphere8_q2": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 8, 2, 2, 120),
}


def _setup(name):
    """GPU build plus the oracle's enumeration and neighbour rows (its stencils only where
    a test needs them)."""
    shape, n, Q, R, nsub = CASES[name]
    g = cg.make_geometry(shape, n, Q)
    en = oracle.enumerate_geometry(g)
    nbr = [oracle.neighbours(en, f, R) for f in range(en.n_face)]
    rp = np.zeros(en.n_face + 1, np.int64)
    rp[1:] = np.cumsum([len(x) for x in nbr])
    col = np.concatenate(nbr).astype(np.int32)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    b = cc.Builder(dg, R)
    st = b.build()
    torch.cuda.synchronize()
    assert np.array_equal(st.row_ptr.cpu().numpy(), rp)
    assert np.array_equal(st.col.cpu().numpy()[: len(col)], col)
    val = st.val.cpu().numpy()[: len(col)]
    return g, en, rp, col, val, R, dg, b, st, nsub


def _face_subset(en, nsub, seed):
    """nsub faces: every EB face and grid face of a few cut cells, plus random others."""
    if nsub is None:
        return np.arange(en.n_face)
    rng = np.random.default_rng(seed)
    eb_faces = np.flatnonzero(en.face_kind == oracle.stencils.KIND_EB)
    owners = set(int(en.face_lo[f]) for f in rng.choice(eb_faces, 3, replace=False))
    near = [f for f in range(en.n_face) if int(en.face_lo[f]) in owners or int(en.face_hi[f]) in owners]
    box = np.flatnonzero((en.face_lo < 0) | (en.face_hi < 0))
    extra = rng.choice(en.n_face, nsub, replace=False)
    sel = np.unique(np.concatenate([near, rng.choice(box, 6, replace=False), rng.choice(eb_faces, 6, replace=False),
                                    extra]))
    return sel


def _val_bar(rp, faces, nnz, seed):
    vb = np.zeros(nnz)
    rng = np.random.default_rng(seed)
    for f in faces:
        vb[rp[f]:rp[f + 1]] = rng.standard_normal(rp[f + 1] - rp[f])
    return vb


def _cmp(name, got, ref, tol=GRAD_TOL):
    got = np.asarray(got)
    ref = np.asarray(ref)
    assert got.shape == ref.shape, (name, got.shape, ref.shape)
    scale = np.abs(ref).max()
    err = np.abs(got - ref).max()
    _say(f"{name}: max|ref| {scale:.3e} max err {err:.3e} rel {err / max(scale, 1e-300):.3e}")
    assert err <= tol * scale + 1e-300, (name, err, scale)


@pytest.mark.parametrize("name", ["circle16_q4", "sphere10_q4"])
def test_apply_adjoint_matches_oracle(name):
    g, en, rp, col, valg, R, dg, b, st, _ = _setup(name)
    _say(f"apply adjoint {name}")
    rng = np.random.default_rng(5)
    phi = rng.standard_normal(en.n_phi)
    lbar = rng.standard_normal(en.n_vol)
    phi_t = torch.from_numpy(phi).to(DEV)
    lphi, flux = cc.apply(st, phi_t)
    phi_bar, val_bar, scale_bar, flux_bar = cc.apply_adjoint(st, torch.from_numpy(lbar).to(DEV), phi=phi_t,
                                                             flux=flux)
    torch.cuda.synchronize()
    pb_o, vb_o, kb_o = oracle.apply_adjoint(g, en, rp, col, valg, phi, lbar)
    # phi_bar: sums over the column's nonzeros of val * flux_bar
    scale = 1.0 / (g.vol_mom[en.vol_cell, 0] * en.h**en.D)
    c = np.zeros(en.n_face)
    for side, sgn in ((en.face_lo, 1.0), (en.face_hi, -1.0)):
        m = side >= 0
        np.add.at(c, np.flatnonzero(m), sgn * lbar[side[m]] * scale[side[m]])
    bound = np.zeros(en.n_phi)
    np.add.at(bound, col, np.abs(valg * c[np.repeat(np.arange(en.n_face), np.diff(rp))]))
    assert np.all(np.abs(phi_bar.cpu().numpy() - pb_o) <= 1e-12 * bound + 1e-300)
    assert np.all(np.abs(val_bar.cpu().numpy() - vb_o) <= 1e-12 * np.abs(vb_o) + 1e-300)
    # scale_bar -> kappa_bar = -scale_bar * scale / kappa
    kap = g.vol_mom[en.vol_cell, 0]
    kb_g = -scale_bar.cpu().numpy() * st.vol_scale.cpu().numpy()[: en.n_vol] / kap
    assert np.all(np.abs(kb_g - kb_o) <= 1e-12 * np.abs(kb_o) + 1e-14 * np.abs(kb_o).max())
    # transpose identity on the device results
    lhs = float(torch.dot(torch.from_numpy(lbar).to(DEV), lphi))
    rhs = float(torch.dot(phi_bar, phi_t))
    assert abs(lhs - rhs) <= 1e-12 * float(torch.dot(torch.from_numpy(np.abs(lbar)).to(DEV), lphi.abs()))


@pytest.mark.parametrize("name", list(CASES))
def test_stencil_gradients_match_oracle(name):
    g, en, rp, col, val, R, dg, b, st, nsub = _setup(name)
    faces = _face_subset(en, nsub, 11)
    _say(f"stencils backward {name}: {len(faces)} of {en.n_face} faces")
    vb = _val_bar(rp, faces, len(col), 12)
    grads, wb = b.backward(st, torch.from_numpy(vb).to(DEV), weight_bar=True)
    torch.cuda.synchronize()
    G = oracle.stencils_backward(g, en, R, rp, vb, faces=faces)
    gg = grads[0]
    _cmp("vol_mom", gg["vol_mom"].cpu().numpy(), G["vol_mom"])
    for d in range(g.D):
        _cmp(f"face_mom[{d}]", gg["face_mom"][d].cpu().numpy(), G["face_mom"][d])
    _cmp("eb_mom", gg["eb_mom"].cpu().numpy(), G["eb_mom"])
    _cmp("eb_nmom", gg["eb_nmom"].cpu().numpy(), G["eb_nmom"])
    _cmp("weight", wb.cpu().numpy(), G["weight"])


def test_stencil_backward_is_deterministic():
    g, en, rp, col, val, R, dg, b, st, _ = _setup("circle16_q4")
    vb = torch.from_numpy(np.random.default_rng(3).standard_normal(len(col))).to(DEV)
    g1, w1 = b.backward(st, vb, weight_bar=True)
    g2, w2 = b.backward(st, vb, weight_bar=True)
    torch.cuda.synchronize()
    assert torch.equal(g1[0]["vol_mom"], g2[0]["vol_mom"])
    assert torch.equal(g1[0]["eb_nmom"], g2[0]["eb_nmom"])
    assert all(torch.equal(a, c) for a, c in zip(g1[0]["face_mom"], g2[0]["face_mom"]))
    assert torch.equal(w1, w2)


def test_batch_backward_equals_separate():
    shapes = [cg.ball_outside((0.5, 0.5), 0.25), cg.ball_outside((0.47, 0.52), 0.27)]
    geoms = [cg.make_geometry(s, 16, 4) for s in shapes]
    dgs = [cc.DeviceGeometry.from_host(h, DEV) for h in geoms]
    bb = cc.Builder(dgs, 3)
    st = bb.build()
    nnz = st.sizes.nnz
    vb = torch.from_numpy(np.random.default_rng(9).standard_normal(nnz)).to(DEV)
    gb, _ = bb.backward(st, vb)
    off = 0
    for i, dg in enumerate(dgs):
        b1 = cc.Builder(dg, 3)
        s1 = b1.build()
        n1 = s1.sizes.nnz
        g1, _ = b1.backward(s1, vb[off: off + n1].contiguous())
        off += n1
        assert torch.equal(g1[0]["vol_mom"], gb[i]["vol_mom"])
        assert torch.equal(g1[0]["eb_mom"], gb[i]["eb_mom"])
        assert all(torch.equal(a, c) for a, c in zip(g1[0]["face_mom"], gb[i]["face_mom"]))
    assert off == nnz


def test_autograd_loss_gradient_matches_oracle():
    """l = sum over cut volumes of (L(Phi) - f)^2 with Phi the exact solution's averages:
    torch.autograd through CutCellOperator vs the oracle's apply adjoint chained into its
    stencil adjoint (including d(1/kappa)/dkappa)."""
    shape = cg.ball_outside((0.5, 0.5), 0.25)
    g = cg.make_geometry(shape, 16, 2)
    R = 2
    en, rp, col, val, status = oracle.build(g, R)
    rng = np.random.default_rng(21)
    phi = rng.standard_normal(en.n_phi)
    f = rng.standard_normal(en.n_vol)
    cut = np.isin(en.vol_cell, g.eb_cell).astype(np.float64)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    for t in [dg.vol_mom, *dg.face_mom, dg.eb_mom, dg.eb_nmom]:
        t.requires_grad_(True)
    op = cc.CutCellOperator(dg, R)
    phi_t = torch.from_numpy(phi).to(DEV).requires_grad_(True)
    L = op(phi_t)
    loss = torch.sum(torch.from_numpy(cut).to(DEV) * (L - torch.from_numpy(f).to(DEV)) ** 2)
    loss.backward()
    torch.cuda.synchronize()
    # oracle chain
    _, L_o = oracle.apply(g, en, rp, col, val, phi)
    lbar = 2 * cut * (L_o - f)
    pb_o, vb_o, kb_o = oracle.apply_adjoint(g, en, rp, col, val, phi, lbar)
    G = oracle.stencils_backward(g, en, R, rp, vb_o, weights=False)
    vol_o = G["vol_mom"].copy()
    np.add.at(vol_o[:, 0], en.vol_cell, kb_o)
    _cmp("phi", phi_t.grad.cpu().numpy(), pb_o)
    _cmp("vol_mom", dg.vol_mom.grad.cpu().numpy(), vol_o)
    for d in range(2):
        _cmp(f"face_mom[{d}]", dg.face_mom[d].grad.cpu().numpy(), G["face_mom"][d])
    _cmp("eb_mom", dg.eb_mom.grad.cpu().numpy(), G["eb_mom"])
    _cmp("eb_nmom", dg.eb_nmom.grad.cpu().numpy(), G["eb_nmom"])


def test_sh_body_128_shape_gradient_by_finite_differences():
    """The differentiation workload: the 128^3 unit cube minus the body
    r = 0.3 + sum_{l<=3} c_lm Y_lm about (0.5, 0.5, 0.5), c = 0.01 * default_rng(4) N(0,1)
    (16 coefficients), order 4, path radius 3.  Loss: l = sum over cut volumes of
    (kappa_v (L_v(Phi) - f_v))^2 with Phi and f fixed vectors, the exact averages at c of the
    paper's 3D solution sin 2pi(x - sqrt2/2) sin 2pi(y - sqrt3/2) sin 2pi(z - 0.54321) and of
    its Laplacian.  The autograd gradient with respect to every moment (through the
    hand-written adjoints), contracted with central differences of the host moments in a
    shape coefficient, must match central differences of the loss itself.  The loss is only
    piecewise smooth in c: a coefficient is used only if between c - h and c + h no cell
    or face changes topology and no face's status changes.  It is also very stiff: the
    residuals r_v = kappa_v (L_v - f_v) are ~1e-5 at c but move ~1e6 times faster than c
    (a face flux is a sum of terms ~5e3 times larger than itself, and near-tangent cuts
    move EB moments quickly), so the central difference of l = sum r^2 carries an error
    sum r' r'' h^2 that swamps sum 2 r r' at h = 1e-7 (it is 1.2e-5 relative at h = 1e-9).
    Both sides are therefore Richardson-extrapolated from h = 2e-9 and 1e-9, which removes
    the h^2 term; the host moments' differences stay accurate to ~1e-7 at these steps.
    Every coefficient is tried; those whose steps change the topology are listed and
    skipped.  The differences carry an absolute error (the loss's rounding and the host
    quadrature, amplified by 1/2h) that does not shrink with a coefficient's derivative, so
    every coefficient is held to 1e-6 of the largest derivative (the gradient's infinity
    norm); each one's own relative error is logged.  The builds solve every face on the Gram path (factorization "gram"): in the
    default mode a face near the routing bounds can take the QR path at c + h and not at
    c - h, a rounding-level change of its stencil that differences at h = 1e-9 of this
    stiff loss would amplify."""
    R, n, Q, hstep = 3, 128, 4, 1e-9
    c0 = 0.01 * np.random.default_rng(4).standard_normal(16)
    shape = lambda c: cg.sh_body_outside((0.5, 0.5, 0.5), 0.3, c)  # noqa: E731
    g = cg.make_geometry(shape(c0), n, Q)
    tp = 2 * np.pi
    field = cg.trig_product((tp, tp, tp), (-tp * np.sqrt(2) / 2, -tp * np.sqrt(3) / 2, -tp * 0.54321))
    I = g.integrate(field)
    en = oracle.enumerate_geometry(g)
    hD, hD1 = g.h**3, g.h**2
    vol = en.vol_cell
    box = np.array([I["face_int"][d][f] / (g.face_mom[d][f, 0] * hD1) for d, f in zip(en.box_dir, en.box_face)])
    phi = np.concatenate([I["vol_int"][vol] / (g.kappa[vol] * hD), I["eb_int"] / (g.eb_mom[:, 0] * hD1), box])
    fvol = I["vol_lap"][vol] / (g.kappa[vol] * hD)
    cut = np.isin(vol, g.eb_cell)
    _say(f"sh body 128^3: {en.n_face} faces, {int(cut.sum())} cut volumes")
    phi_t = torch.from_numpy(phi).to(DEV)
    f_t = torch.from_numpy(fvol).to(DEV)
    cut_t = torch.from_numpy(cut).to(DEV)
    cells_t = torch.from_numpy(vol.astype(np.int64)).to(DEV)

    def loss_of(dg, keep=None):
        op = cc.CutCellOperator(dg, R, factorization="gram")
        L = op(phi_t)
        kap = dg.vol_mom[:, 0][cells_t]
        r = torch.where(cut_t, kap * (L - f_t), torch.zeros_like(L))
        if keep is not None:
            keep.append(op.builder.last.status[: op.builder.last.sizes.n_face].clone())
        return torch.sum(r * r)

    dg = cc.DeviceGeometry.from_host(g, DEV)
    leaves = [dg.vol_mom, *dg.face_mom, dg.eb_mom, dg.eb_nmom]
    for t in leaves:
        t.requires_grad_(True)
    st0 = []
    loss = loss_of(dg, st0)
    loss.backward()
    nflag = int((st0[0] != 0).sum())
    torch.cuda.synchronize()
    grads = [t.grad.cpu().numpy() for t in leaves]
    _say(f"loss {float(loss.detach()):.6e}, {nflag} faces flagged")

    def arrays(gg):
        return [gg.vol_mom, *gg.face_mom, gg.eb_mom, gg.eb_nmom]

    def same_topology(gg):
        return (np.array_equal(gg.eb_cell, g.eb_cell) and np.array_equal(gg.kappa > 0, g.kappa > 0)
                and all(np.array_equal(gg.face_mom[d][:, 0] > 0, g.face_mom[d][:, 0] > 0) for d in range(3)))

    def central(k, hh):
        """(adjoint contracted with the moments' central difference, central difference of
        l) at step hh, or None when the topology or a status changes within +-hh."""
        cp, cm = c0.copy(), c0.copy()
        cp[k] += hh
        cm[k] -= hh
        gp, gm = cg.make_geometry(shape(cp), n, Q), cg.make_geometry(shape(cm), n, Q)
        if not (same_topology(gp) and same_topology(gm)):
            return None
        stp, stm = [], []
        with torch.no_grad():
            lp = float(loss_of(cc.DeviceGeometry.from_host(gp, DEV), stp))
            lm = float(loss_of(cc.DeviceGeometry.from_host(gm, DEV), stm))
        if not (torch.equal(stp[0], st0[0]) and torch.equal(stm[0], st0[0])):
            return None
        dmu = [(x - y) / (2 * hh) for x, y in zip(arrays(gp), arrays(gm))]
        adj = sum(float(np.sum(gr * dm)) for gr, dm in zip(grads, dmu))
        return adj, (lp - lm) / (2 * hh)

    checked, skipped, results = [], [], []
    for k in range(16):
        r1 = central(k, 2 * hstep)
        r2 = central(k, hstep) if r1 is not None else None
        if r2 is None:
            _say(f"coefficient {k}: topology or a status changes within the steps; not differentiable here")
            skipped.append(k)
            continue
        checked.append(k)
        # Richardson: the O(h^2) terms of both central differences cancel
        adj = (4 * r2[0] - r1[0]) / 3
        fd = (4 * r2[1] - r1[1]) / 3
        _say(f"coefficient {k}: h={2 * hstep:g}: adjoint {r1[0]:.10e} fd {r1[1]:.10e}; h={hstep:g}: adjoint "
             f"{r2[0]:.10e} fd {r2[1]:.10e}")
        _say(f"coefficient {k}: extrapolated adjoint {adj:.10e}  finite difference {fd:.10e}  "
             f"rel {abs(adj - fd) / abs(fd):.2e}")
        results.append((k, adj, fd))
    scale = max(abs(fd) for _, _, fd in results)
    worst = max(abs(adj - fd) for _, adj, fd in results) / scale
    _say(f"shape coefficients checked: {len(checked)} of 16 {checked}; skipped (topology changes within "
         f"the steps): {skipped}; worst |adjoint - fd| / max|fd| {worst:.2e}")
    for k, adj, fd in results:
        assert abs(adj - fd) <= 1e-6 * scale, (k, adj, fd, scale)
    assert len(checked) >= 8, "too few shape coefficients keep the topology within +-h"


def test_sh_body_128_gradients_match_oracle():
    """The differentiation workload's stencil adjoint at full size (128^3, 5.7M faces)
    against the oracle's: val_bar drawn on a seeded subset of faces -- every face of the 4
    smallest cut cells, 40 faces next to cut cells and 20 random faces -- and zero elsewhere
    (the gradient of every other face is then zero on both sides); every moment gradient
    at the 1e-9 bar of the small cases."""
    R, n, Q = 3, 128, 4
    c0 = 0.01 * np.random.default_rng(4).standard_normal(16)
    g = cg.make_geometry(cg.sh_body_outside((0.5, 0.5, 0.5), 0.3, c0), n, Q)
    en = oracle.enumerate_geometry(g)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    b = cc.Builder(dg, R)
    st = b.build()
    torch.cuda.synchronize()
    rp = st.row_ptr.cpu().numpy()
    rng = np.random.default_rng(31)
    kap = g.kappa[en.vol_cell]
    cut = np.zeros(en.n_vol, bool)
    cut[en.vol_of_cell[en.eb_cell]] = True
    small = np.argsort(np.where(cut, kap, np.inf))[:4]
    lo, hi = en.face_lo, en.face_hi
    of_small = np.flatnonzero(np.isin(lo, small) | np.isin(hi, small))
    near = np.flatnonzero(((lo >= 0) & cut[np.maximum(lo, 0)]) | ((hi >= 0) & cut[np.maximum(hi, 0)]))
    faces = np.unique(np.concatenate([of_small, rng.choice(near, 40, replace=False),
                                      rng.choice(en.n_face, 20, replace=False)]))
    _say(f"sh body 128^3 adjoint vs oracle: {len(faces)} faces (smallest cut cell kappa {kap[small[0]]:.2e})")
    vb = np.zeros(int(st.sizes.nnz))
    for f in faces:
        vb[rp[f]:rp[f + 1]] = rng.standard_normal(rp[f + 1] - rp[f])
    grads, _ = b.backward(st, torch.from_numpy(vb).to(DEV))
    torch.cuda.synchronize()
    G = oracle.stencils_backward(g, en, R, rp, vb, faces=faces, weights=False)
    gg = grads[0]
    _cmp("128^3 vol_mom", gg["vol_mom"].cpu().numpy(), G["vol_mom"])
    for d in range(3):
        _cmp(f"128^3 face_mom[{d}]", gg["face_mom"][d].cpu().numpy(), G["face_mom"][d])
    _cmp("128^3 eb_mom", gg["eb_mom"].cpu().numpy(), G["eb_mom"])
    _cmp("128^3 eb_nmom", gg["eb_nmom"].cpu().numpy(), G["eb_nmom"])
