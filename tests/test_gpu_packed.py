"""Compressed stencils (cutcell_pack_*, cutcell_apply_packed): a face whose stencil was
copied from a template face is stored as the template's slot plus one Phi index per run
of consecutive columns.  The packed apply must give cutcell_apply's flux and L(Phi) bit
for bit, so every test compares the two with torch.equal."""

import numpy as np
import pytest

import cutgeom as cg

torch = pytest.importorskip("torch")
import paper_1411_4283_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _build(geoms, R, **kw):
    dg = [cc.DeviceGeometry.from_host(g, DEV) for g in geoms]
    st = cc.Builder(dg, R, **kw).build()
    torch.cuda.synchronize()
    return st


def _phi(st, seed):
    rng = np.random.default_rng(seed)
    return torch.from_numpy(rng.standard_normal(st.sizes.n_phi)).to(DEV)


def _check(st, label, seed=5):
    pk = cc.pack(st)
    phi = _phi(st, seed)
    lphi, flux = cc.apply(st, phi)
    lphi2, flux2 = cc.apply_packed(st, pk, phi)
    torch.cuda.synchronize()
    n = int(pk.sizes.n_packed)
    _say(f"{label}: {st.sizes.n_face} faces, {st.reused} copied, {n} packed in {pk.sizes.n_slot} slots "
         f"(<= {pk.sizes.max_runs} runs of {pk.sizes.max_rows} rows)")
    assert torch.equal(flux, flux2), f"{label}: flux differs"
    assert torch.equal(lphi, lphi2), f"{label}: L(phi) differs"
    return pk


def test_full_size_sphere_packs_every_copy_and_is_bitwise():
    """The 64^3 fourth-order workload: every template copy packs, L(phi) is bitwise."""
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 64, 4)
    st = _build([g], 3, reuse_templates=True)
    pk = _check(st, "sphere64")
    assert st.reused > st.sizes.n_face // 3
    assert int(pk.sizes.n_packed) == st.reused
    flag = pk.flag[: st.sizes.n_face].to(torch.int64)
    tmpl = st.tmpl[: st.sizes.n_face]
    assert torch.equal(flag.bool(), tmpl >= 0)
    # packed faces ascending; their run bases reproduce the CSR columns; the phases are
    # the row offsets within the flux pass's 4-face groups
    face = pk.face[: int(pk.sizes.n_packed)].to(torch.int64)
    assert bool((face[1:] > face[:-1]).all())
    rp = st.row_ptr.cpu().numpy()
    f_all = np.arange(st.sizes.n_face)
    assert np.array_equal(pk.phase[: st.sizes.n_face].cpu().numpy(), (rp[f_all] - rp[f_all - f_all % 4]) % 64)
    col = st.col.cpu().numpy()
    fc = face.cpu().numpy()
    slot = pk.slot.cpu().numpy()
    base = pk.base.cpu().numpy().reshape(-1, pk.sizes.max_runs)
    tab = pk.slot_tab.cpu().numpy().reshape(-1, pk.sizes.max_rows)
    for i in np.random.default_rng(1).choice(len(fc), 200, replace=False):
        f = fc[i]
        n = rp[f + 1] - rp[f]
        t = tab[slot[i], :n]
        rebuilt = base[i, t & 0xFFFF] + (t >> 16)
        assert np.array_equal(rebuilt, col[rp[f]:rp[f + 1]]), f


def test_batch_neumann_and_2d():
    gs = [cg.make_geometry(cg.ball_outside((0.5 + 0.01 * k, 0.5, 0.5), 0.25 + 0.02 * k), 32, 4) for k in range(3)]
    st = _build(gs, 3, reuse_templates=True)
    pk = _check(st, "batch of three spheres")
    assert int(pk.sizes.n_slot) == 9 and int(pk.sizes.n_packed) == st.reused
    stn = _build(gs, 3, reuse_templates=True, eb_bc="neumann")
    _check(stn, "same batch, Neumann")
    g2 = cg.make_geometry(cg.star2_outside((0.5, 0.5), 0.25, 0.05, 6), 128, 4)
    st2 = _build([g2], 3, reuse_templates=True)
    pk2 = _check(st2, "star128 (2D)")
    assert int(pk2.sizes.n_packed) == st2.reused > 0
    g3 = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.3), 64, 2)
    _check(_build([g3], 2, reuse_templates=True), "circle64 order 2 (2D)")


def test_without_reuse_nothing_packs():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 24, 4)
    st = _build([g], 3)
    assert bool((st.tmpl[: st.sizes.n_face] == -1).all())
    pk = _check(st, "sphere24 without reuse")
    assert int(pk.sizes.n_packed) == 0 and int(pk.sizes.n_slot) == 0


def test_a_face_whose_row_differs_from_its_template_is_not_packed():
    """Point faces at templates whose rows they do not reproduce (other row counts or
    values): the pack must keep them as CSR rows (the apply stays bitwise); faces pointed
    at their true template still pack."""
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 32, 4)
    st = _build([g], 3, reuse_templates=True)
    nf = st.sizes.n_face
    tmpl = st.tmpl[:nf].clone()
    copies = torch.nonzero(tmpl >= 0).flatten()
    assert len(copies) > 0
    t0 = int(tmpl[copies[0]])
    rp = st.row_ptr.cpu().numpy()
    val = st.val.cpu().numpy()
    row_t = val[rp[t0]:rp[t0 + 1]]
    solved = torch.nonzero(tmpl < 0).flatten().cpu().numpy()
    victims = []
    for f in solved[:: max(1, len(solved) // 400)]:
        row = val[rp[f]:rp[f + 1]]
        if f != t0 and (len(row) != len(row_t) or not np.array_equal(row.view(np.int64), row_t.view(np.int64))):
            victims.append(int(f))
    victims = torch.tensor(victims[:50], dtype=torch.int64, device=DEV)
    assert len(victims) == 50
    st.tmpl[victims] = t0
    pk = _check(st, "sphere32 with false templates")
    flag = pk.flag[:nf].bool()
    assert not bool(flag[victims].any())
    assert int(pk.sizes.n_packed) == len(copies)


def test_empty_batch():
    g = cg.make_geometry(cg.halfspace([0.0, 1.0], 2.0), 16, 4)   # fluid nowhere in the box
    st = _build([g], 3, reuse_templates=True)
    assert st.sizes.n_face == 0
    pk = cc.pack(st)
    assert int(pk.sizes.n_packed) == 0
    L, flux = cc.apply_packed(st, pk, torch.zeros(0, dtype=torch.float64, device=DEV))
    assert L.numel() == 0 and flux.numel() == 0
