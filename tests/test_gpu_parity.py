"""GPU parity: the HIP library through its C ABI against the CPU oracle.

Bars (written in each test):
  * row_ptr, col and status bit-exact;
  * stencil values per face: max|s_gpu - s_orc| <= 1e-11 * max|s_orc| (flat: the oracle
    computes in extended precision, its own error stays below 1e-12 up to cond ~1e7, and
    faces the Gram path cannot resolve to this bar are solved by Householder QR);
  * L(Phi) on the same stencils: per volume |dL_v| <= 1e-12 * sum_f sum_j |s_fj Phi_j| / |V_v|
    and ||dL||_2 <= 1e-12 ||L||_2.
Small cases are compared entry by entry; the full-size 64^3 workload on sampled faces
and through properties that hold at any size.
"""

import numpy as np
import pytest

import cutgeom as cg
import oracle
from oracle import stencils as S

torch = pytest.importorskip("torch")
import paper_1411_4283_amd as cc  # noqa: E402

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _say(msg):
    print(f"[gpu] {msg}", flush=True)


def _gpu_build(g, R):
    dg = cc.DeviceGeometry.from_host(g, DEV)
    b = cc.Builder(dg, R)
    st = b.build()
    torch.cuda.synchronize()
    return dg, b, st


def _host(st):
    s = st.sizes
    return (st.row_ptr.cpu().numpy(), st.col.cpu().numpy()[: s.nnz], st.val.cpu().numpy()[: s.nnz],
            st.status.cpu().numpy()[: s.n_face])


def _check_faces(g, en, R, faces, rp_g, col_g, val_g, st_g, where=None):
    """Compare the listed faces with the oracle, one by one; `where` (a list) receives
    (error, face) of the worst one."""
    worst = 0.0
    for f in faces:
        f = int(f)
        idx, s, status = oracle.face_stencil(g, en, f, R)
        a, b = rp_g[f], rp_g[f + 1]
        assert b - a == len(idx), f"face {f}: {b - a} rows vs {len(idx)}"
        assert np.array_equal(col_g[a:b], idx), f"face {f}: neighbour indices differ"
        assert st_g[f] == status, f"face {f}: status {st_g[f]} vs {status}"
        if status != oracle.STATUS_OK:
            assert np.all(val_g[a:b] == 0)
            continue
        err = np.abs(val_g[a:b] - s).max() / np.abs(s).max()
        assert err <= 1e-11, f"face {f}: rel err {err:.3e}, cond {oracle.face_condition(g, en, f, R):.3e}"
        if where is not None and err > worst:
            where[:] = [err, f]
        worst = max(worst, err)
    return worst


def _check_apply(g, en, st, rp, col, val, phi, norm_check=True):
    """L(Phi) from the GPU against the oracle's apply of the same stencils.  The per-volume
    bound is the rounding bound of the sums (relative to the sum of the magnitudes of the
    terms).  The norm-wise bound ||dL|| <= 1e-12 ||L|| only applies when L is not itself a
    small difference of large fluxes (random Phi); for smooth fields L_v cancels the fluxes
    down by 1/(kappa h^D) and only the per-volume bound is meaningful (norm_check=False)."""
    lphi, flux = cc.apply(st, torch.from_numpy(phi).to(DEV))
    torch.cuda.synchronize()
    Lg = lphi.cpu().numpy()
    fg = flux.cpu().numpy()
    f_o, L_o = oracle.apply(g, en, rp, col, val, phi)
    absterm = np.array([np.abs(val[rp[f]:rp[f + 1]]) @ np.abs(phi[col[rp[f]:rp[f + 1]]]) for f in range(en.n_face)])
    assert np.all(np.abs(fg - f_o) <= 1e-12 * absterm + 1e-300)
    scale = np.zeros(en.n_vol)
    for side in (en.face_lo, en.face_hi):
        m = side >= 0
        np.add.at(scale, side[m], absterm[m])
    scale /= g.kappa[en.vol_cell] * g.h**g.D
    assert np.all(np.abs(Lg - L_o) <= 1e-12 * scale)
    if norm_check:
        assert np.linalg.norm(Lg - L_o) <= 1e-12 * np.linalg.norm(L_o)
    return Lg


CASES = {
    # name: (shape, n, Q, R)
    "circle32_q2": (cg.ball_outside((0.5, 0.5), 0.25), 32, 2, 2),
    "circle32_q4": (cg.ball_outside((0.5, 0.5), 0.25), 32, 4, 3),
    "star64_q4": (cg.star2_outside((0.5, 0.5), 0.25, 0.05, 6), 64, 4, 3),
    "sphere12_q4": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 12, 4, 3),
    "sphere10_q2": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 10, 2, 2),
}


@pytest.mark.parametrize("name", list(CASES))
def test_full_parity(name):
    shape, n, Q, R = CASES[name]
    _say(f"full parity {name}")
    g = cg.make_geometry(shape, n, Q)
    dg, b, st = _gpu_build(g, R)
    en, rp, col, val, status = oracle.build(g, R)
    s = st.sizes
    assert (s.n_vol, s.n_eb, s.n_box, s.n_phi, s.n_face, s.nnz) == (en.n_vol, en.n_eb, en.n_box, en.n_phi,
                                                                   en.n_face, len(col))
    assert s.max_rows == np.diff(rp).max()
    rp_g, col_g, val_g, st_g = _host(st)
    assert np.array_equal(rp_g, rp)
    assert np.array_equal(col_g, col)
    assert np.array_equal(st_g, status)
    worst = 0.0
    for f in range(en.n_face):
        a, b = rp[f], rp[f + 1]
        if status[f] != oracle.STATUS_OK:
            assert np.all(val_g[a:b] == 0)
            continue
        err = np.abs(val_g[a:b] - val[a:b]).max() / np.abs(val[a:b]).max()
        assert err <= 1e-11, f"face {f}: rel err {err:.3e}, cond {oracle.face_condition(g, en, f, R):.3e}"
        worst = max(worst, err)
    _say(f"{name}: {en.n_face} faces, worst stencil rel err {worst:.2e}, {st.qr_faces} by QR")
    phi = np.random.default_rng(5).standard_normal(en.n_phi)
    _check_apply(g, en, st, rp_g, col_g, val_g, phi)


@pytest.fixture(scope="module")
def c3():
    """The 3D fourth-order workload at full size: 64^3 cube minus the r = 0.3 sphere."""
    _say("c3 build")
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 64, 4)
    dg, b, st = _gpu_build(g, 3)
    en = oracle.enumerate_geometry(g)
    return g, en, dg, b, st


def test_full_size_counts_and_sampled_faces(c3):
    g, en, dg, b, st = c3
    s = st.sizes
    assert (s.n_vol, s.n_eb, s.n_box, s.n_phi, s.n_face) == (en.n_vol, en.n_eb, en.n_box, en.n_phi, en.n_face)
    rp_g, col_g, val_g, st_g = _host(st)
    assert rp_g[-1] == s.nnz
    assert np.all(st_g == oracle.STATUS_OK)
    rng = np.random.default_rng(9)
    faces = np.concatenate([rng.choice(en.n_face, 300, replace=False), np.nonzero(en.face_kind == S.KIND_EB)[0][::60],
                            np.nonzero(en.face_kind == S.KIND_BOX)[0][::500], [0, en.n_face - 1]])
    worst = _check_faces(g, en, 3, faces, rp_g, col_g, val_g, st_g)
    _say(f"c3 sampled {len(faces)} faces, worst rel err {worst:.2e}")


def _targeted_faces(g, en, R, rng, n_small=50, n_cond=50, n_cand=600, n_rand=100, n_cells=5):
    """Faces where the solves are hardest: those of the n_small smallest cut cells (their
    EB face and grid faces), the n_cond worst-conditioned among n_cand seeded candidates
    next to the boundary (EB faces and faces of cut cells), every face of the n_cells
    smallest cells, and n_rand random faces.  Returns (faces, cond of the candidates)."""
    kap = g.kappa[en.vol_cell]
    cut = np.zeros(en.n_vol, bool)
    cut[en.vol_of_cell[en.eb_cell]] = True
    order = np.argsort(np.where(cut, kap, np.inf))
    lo, hi = en.face_lo, en.face_hi

    def faces_of(vols):
        m = np.isin(lo, vols) | np.isin(hi, vols)
        return np.flatnonzero(m)

    small = faces_of(order[:n_small])[: 2 * n_small]
    cells = faces_of(order[:n_cells])
    near = np.flatnonzero(((lo >= 0) & cut[np.maximum(lo, 0)]) | ((hi >= 0) & cut[np.maximum(hi, 0)]))
    cand = rng.choice(near, min(n_cand, len(near)), replace=False)
    conds = np.array([oracle.face_condition(g, en, int(f), R) for f in cand])
    worst = cand[np.argsort(conds)[-n_cond:]]
    rand = rng.choice(en.n_face, n_rand, replace=False)
    return np.unique(np.concatenate([small, worst, cells, rand])), conds


def test_full_size_targeted_faces(c3):
    """The 50 smallest cut cells' faces, the 50 worst-conditioned of 600 faces next to the
    boundary, every face of the 5 smallest cells and 100 random faces, at the flat bar."""
    g, en, dg, b, st = c3
    rp_g, col_g, val_g, st_g = _host(st)
    faces, conds = _targeted_faces(g, en, 3, np.random.default_rng(12))
    worst = _check_faces(g, en, 3, faces, rp_g, col_g, val_g, st_g)
    _say(f"c3 targeted: {len(faces)} faces, cond of candidates up to {conds.max():.2e} (p99 "
         f"{np.percentile(conds, 99):.2e}), worst rel err {worst:.2e}; {st.qr_faces} faces by QR")


def test_full_size_rows_bit_exact(c3):
    """row_ptr and col of every face of the 64^3 workload equal the oracle's rows (Sec. 2.4),
    computed for all faces at once by sparse reachability."""
    g, en, dg, b, st = c3
    rp, col = oracle.neighbours_all(en, 3)
    rp_g = st.row_ptr.cpu().numpy()
    assert np.array_equal(rp_g, rp)
    assert np.array_equal(st.col[: st.sizes.nnz].cpu().numpy().astype(np.int64), col)
    _say(f"c3 rows: {en.n_face} faces, {len(col)} entries bit-exact")


def test_batched_perturbed_spheres_against_oracle():
    """The batched workload (64 spheres at 48^3, centres 0.5 + U(-0.05,0.05)^3, radii
    U(0.25,0.35), default_rng(3)): eight of its geometries (seeded choice) built as one batch,
    and in each the faces of the 50 smallest cut cells, the 50 worst-conditioned of 400
    boundary faces, every face of the 5 smallest cells and 100 random faces against the
    oracle at the flat bar; row counts of every face of the batch against the oracle's."""
    shapes = cg.perturbed_spheres(64, 3)
    pick = sorted(np.random.default_rng(21).choice(64, 8, replace=False).tolist())
    gs = [cg.make_geometry(shapes[i], 48, 4) for i in pick]
    _say(f"c4 subset {pick}")
    dgs = [cc.DeviceGeometry.from_host(g, DEV) for g in gs]
    st = cc.Builder(dgs, 3).build()
    torch.cuda.synchronize()
    fo, po = st.face_off.cpu().numpy(), st.phi_off.cpu().numpy()
    rpb = st.row_ptr.cpu().numpy()
    colb = st.col[: st.sizes.nnz].cpu().numpy()
    valb = st.val[: st.sizes.nnz].cpu().numpy()
    stsb = st.status[: st.sizes.n_face].cpu().numpy()
    worst_all, conds_all, worst_at = 0.0, [], None
    for k, g in enumerate(gs):
        en = oracle.enumerate_geometry(g)
        a, e = fo[k], fo[k + 1]
        rp_g = rpb[a:e + 1] - rpb[a]
        col_g = colb[rpb[a]:rpb[e]] - po[k]
        val_g = valb[rpb[a]:rpb[e]]
        rp_o, _ = oracle.neighbours_all(en, 3)
        assert np.array_equal(rp_g, rp_o)
        faces, conds = _targeted_faces(g, en, 3, np.random.default_rng(100 + k), n_cand=400)
        where = []
        w = _check_faces(g, en, 3, faces, rp_g, col_g, val_g, stsb[a:e], where)
        if w > worst_all:
            worst_all = w
            worst_at = (k, where[1], oracle.face_condition(g, en, where[1], 3))
        conds_all.append(conds)
    c = np.concatenate(conds_all)
    _say(f"c4: {len(gs)} geometries, {st.sizes.n_face} faces, {st.qr_faces} by QR; candidate cond p50 "
         f"{np.median(c):.2e} p99 {np.percentile(c, 99):.2e} max {c.max():.2e}; worst rel err {worst_all:.2e} "
         f"(geometry {worst_at[0]}, face {worst_at[1]}, cond {worst_at[2]:.2e})")


def test_full_size_faces_of_every_row_count_in_the_split_bin(c3):
    """The 96-row bin of this workload runs as two launches: faces with at most 88 rows on
    an 88-row kernel instance, the rest on the 96-row one.  Three seeded faces of every
    row count from 81 to 96 (both launches, both sides of the boundary) against the oracle."""
    g, en, dg, b, st = c3
    rp_g, col_g, val_g, st_g = _host(st)
    n = np.diff(rp_g)
    rng = np.random.default_rng(11)
    faces, seen = [], []
    for rows in range(81, 97):
        cand = np.nonzero(n == rows)[0]
        if len(cand):
            seen.append(rows)
            faces.extend(rng.choice(cand, min(3, len(cand)), replace=False))
    assert any(r <= 88 for r in seen) and any(r > 88 for r in seen)
    worst = _check_faces(g, en, 3, faces, rp_g, col_g, val_g, st_g)
    _say(f"c3 split bin: {len(faces)} faces with {seen[0]}..{seen[-1]} rows, worst rel err {worst:.2e}")


def test_full_size_rows_sorted_and_in_range(c3):
    g, en, dg, b, st = c3
    rp_g, col_g, val_g, st_g = _host(st)
    N = np.diff(rp_g)
    assert N.min() >= 35 and N.max() <= 128
    inner = np.ones(len(col_g), bool)
    inner[rp_g[1:] - 1] = False                     # last entry of each row
    assert np.all(col_g[:-1][inner[:-1]] < col_g[1:][inner[:-1]])
    assert col_g.min() >= 0 and col_g.max() < en.n_phi


def test_full_size_polynomial_exactness(c3):
    """Property at any size: every face flux of a random quartic is exact (A^T s = F),
    against an independent quadrature of the same polynomial."""
    g, en, dg, b, st = c3
    pf = cg.random_polynomial(3, 4, np.random.default_rng(2), scale=0.25)
    I = g.integrate(pf)
    hD, hD1 = g.h**3, g.h**2
    vol = en.vol_cell
    box = np.array([I["face_int"][d][f] / (g.face_mom[d][f, 0] * hD1) for d, f in zip(en.box_dir, en.box_face)])
    phi = np.concatenate([I["vol_int"][vol] / (g.kappa[vol] * hD), I["eb_int"] / (g.eb_mom[:, 0] * hD1), box])
    lphi, flux = cc.apply(st, torch.from_numpy(phi).to(DEV))
    fg = flux.cpu().numpy()
    ref = np.empty(en.n_face)
    grid = en.face_kind != S.KIND_EB
    for d in range(3):
        m = grid & (en.face_dir == d)
        ref[m] = I["face_flux"][d][en.face_lin[m]]
    ref[~grid] = I["eb_flux"][en.face_lin[~grid]]
    rp_g, col_g, val_g, _ = _host(st)
    absterm = np.add.reduceat(np.abs(val_g) * np.abs(phi[col_g]), rp_g[:-1])
    assert np.all(np.abs(fg - ref) <= 1e-11 * (absterm + np.abs(ref)))


def test_full_size_apply(c3):
    g, en, dg, b, st = c3
    rp_g, col_g, val_g, _ = _host(st)
    phi = np.random.default_rng(2).standard_normal(en.n_phi)
    _say("c3 apply vs oracle")
    _check_apply(g, en, st, rp_g, col_g, val_g, phi)


def test_build_is_deterministic(c3):
    g, en, dg, b, st = c3
    st2 = b.build()
    torch.cuda.synchronize()
    assert torch.equal(st.row_ptr, st2.row_ptr) and torch.equal(st.col, st2.col)
    assert torch.equal(st.val.view(torch.int64), st2.val.view(torch.int64))


def test_batch_equals_separate_builds():
    _say("batch of three circles")
    shapes = [cg.ball_outside((0.5, 0.5), 0.25), cg.ball_outside((0.51, 0.5), 0.25), cg.ball_outside((0.5, 0.5), 0.255)]
    gs = [cg.make_geometry(s, 32, 4) for s in shapes]
    dgs = [cc.DeviceGeometry.from_host(g, DEV) for g in gs]
    stb = cc.Builder(dgs, 3).build()
    torch.cuda.synchronize()
    po, fo = stb.phi_off.cpu().numpy(), stb.face_off.cpu().numpy()
    rpb, colb, valb, stsb = _host(stb)
    for i, dg in enumerate(dgs):
        st1 = cc.Builder(dg, 3).build()
        rp1, col1, val1, sts1 = _host(st1)
        a, bnd = fo[i], fo[i + 1]
        assert np.array_equal(rpb[a:bnd + 1] - rpb[a], rp1)
        assert np.array_equal(colb[rpb[a]:rpb[bnd]] - po[i], col1)
        assert np.array_equal(valb[rpb[a]:rpb[bnd]].view(np.int64), val1.view(np.int64))
        assert np.array_equal(stsb[a:bnd], sts1)


def test_insufficient_rows_flagged():
    _say("insufficient rows")
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.25), 16, 4)
    dg, b, st = _gpu_build(g, 1)
    assert st.code == 1   # CUTCELL_W_FLAGGED_FACES
    rp, col, val, sts = _host(st)
    assert np.all(sts == oracle.STATUS_INSUFFICIENT_ROWS) and np.all(val == 0)


def test_rank_deficient_and_nonfinite_flagged():
    from test_oracle import _channel_geometry

    _say("rank deficient channel")
    g = _channel_geometry()
    dg, b, st = _gpu_build(g, 3)
    en, rp, col, val, status = oracle.build(g, 3)
    rp_g, col_g, val_g, st_g = _host(st)
    assert np.array_equal(col_g, col) and np.array_equal(st_g, status) and np.all(val_g == 0)

    _say("non-finite moment")
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.25), 16, 2)
    en = oracle.enumerate_geometry(g)
    g.vol_mom[int(en.vol_cell[40]), 3] = np.nan
    dg, b, st = _gpu_build(g, 2)
    en, rp, col, val, status = oracle.build(g, 2)
    rp_g, col_g, val_g, st_g = _host(st)
    assert np.array_equal(st_g, status)
    ok = status == oracle.STATUS_OK
    assert np.any(~ok) and np.any(ok)


def test_bad_eb_cells_rejected():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.25), 16, 2)
    dg = cc.DeviceGeometry.from_host(g, DEV)
    dg.eb_cell = dg.eb_cell.flip(0).contiguous()    # not ascending
    with pytest.raises(cc.CutcellError) as e:
        cc.Builder(dg, 2).query()
    assert e.value.code == -1


def test_every_schedule_gives_identical_stencils():
    """The launch schedule (faces in bin order or in per-XCD chunks, one workgroup per
    face or a persistent grid) changes only which workgroup takes a face: val and status
    must be bit-identical to the default build, and the autotuned build as well."""
    from paper_1411_4283_amd._lib import Tuning

    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 24, 4)
    dg, b, st0 = _gpu_build(g, 3)
    val0, status0 = st0.val.clone(), st0.status.clone()
    for xcd, per, split in [(8, 0, 0), (8, 16, 1), (8, 100, 2), (1, 64, 3), (3, 5, 1), (1, 0, 2)]:
        t = Tuning()
        for i in range(8):
            t.xcd_chunks[i], t.blocks_per_xcd[i], t.split[i] = xcd, per, split
        b.set_tuning(t)
        _say(f"schedule xcd={xcd} per={per} split={split}")
        st = b.build()
        torch.cuda.synchronize()
        assert torch.equal(st.val, val0) and torch.equal(st.status, status0), (xcd, per, split)
    b.set_tuning(None)
    tuning, best = b.autotune()
    st = b.build()
    torch.cuda.synchronize()
    _say(f"autotuned {[(tuning.xcd_chunks[i], tuning.blocks_per_xcd[i], tuning.split[i]) for i in range(8)]} "
         f"best {best}")
    assert torch.equal(st.val, val0) and torch.equal(st.status, status0)
    assert any(x > 0 for x in best)


def test_autotune_cache_round_trip(tmp_path):
    """The JSON cache: a first autotune times every bin and stores each filled bin under
    (arch, D, Q, R, bin); a second one, on another builder of the same shape, takes those
    entries without timing and builds the same stencils."""
    import json

    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 24, 4)
    dg, b, st0 = _gpu_build(g, 3)
    path = str(tmp_path / "tuning.json")
    t1, best1 = b.autotune(cache=path)
    assert not b.tuned_from_cache
    entries = json.load(open(path))
    filled = [i for i in range(8) if best1[i] >= 0]
    assert filled and all(any(k.endswith(f"/D3/Q4/R3/bin{i}") for k in entries) for i in filled)
    b2 = cc.Builder(dg, 3)
    t2, best2 = b2.autotune(cache=path)
    assert b2.tuned_from_cache and best2 == [-1.0] * 8
    for i in filled:
        assert (t2.xcd_chunks[i], t2.blocks_per_xcd[i], t2.split[i]) == (t1.xcd_chunks[i], t1.blocks_per_xcd[i],
                                                                          t1.split[i])
    st = b2.build()
    torch.cuda.synchronize()
    assert torch.equal(st.val, st0.val) and torch.equal(st.status, st0.status)
    _say(f"cache: {len(entries)} entries, bins {filled} reused")


def test_star256_order4_full_size():
    """The 2D fourth-order workload: the unit square minus the six-petal star
    r(t) = 0.25 + 0.05 cos 6t about (0.5, 0.5) on 256^2 (about 106k faces), path radius 3.
    Every face's rows are compared bit-exactly with the oracle's neighbour sets; the
    stencils of every EB face and of 400 seeded random faces with the oracle's; and L(Phi)
    of the seeded Fourier field (modes up to 4, default_rng(1)) with the oracle's apply of
    the same stencils."""
    R = 3
    g = cg.make_geometry(cg.star2_outside((0.5, 0.5), 0.25, 0.05, 6), 256, 4)
    dg, b, st = _gpu_build(g, R)
    en = oracle.enumerate_geometry(g)
    rp_g, col_g, val_g, st_g = _host(st)
    _say(f"star256: {en.n_face} faces, nnz {len(col_g)}")
    assert st.sizes.n_face == en.n_face and st.sizes.n_phi == en.n_phi
    rp, col = oracle.neighbours_all(en, R)
    assert np.array_equal(rp_g, rp)
    assert np.array_equal(col_g, col)
    eb_faces = np.flatnonzero(en.face_kind == S.KIND_EB)
    faces = np.unique(np.concatenate([eb_faces, np.random.default_rng(5).choice(en.n_face, 400, replace=False)]))
    worst = _check_faces(g, en, R, faces, rp_g, col_g, val_g, st_g)
    _say(f"star256: {len(faces)} faces compared, worst stencil rel err {worst:.2e}")
    field = cg.fourier_field(2, 4, np.random.default_rng(1))
    I = g.integrate(field)
    hD, hD1 = g.h**2, g.h
    vol = en.vol_cell
    box = np.array([I["face_int"][d][f] / (g.face_mom[d][f, 0] * hD1) for d, f in zip(en.box_dir, en.box_face)])
    phi = np.concatenate([I["vol_int"][vol] / (g.kappa[vol] * hD), I["eb_int"] / (g.eb_mom[:, 0] * hD1), box])
    _check_apply(g, en, st, rp_g, col_g, val_g, phi, norm_check=False)
