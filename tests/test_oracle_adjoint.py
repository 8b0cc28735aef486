"""Pins for the oracle's adjoints: the transpose identity of the linear apply, and
central finite differences of the numpy forward oracle for the stencil gradients
(the adjoint oracle differentiates an independent torch transcription of the
definition, so agreement pins both)."""

import copy

import numpy as np
import pytest

import cutgeom as cg
import oracle
from oracle import stencils as S

CIRCLE = cg.ball_outside((0.5, 0.5), 0.25)
SPHERE = cg.ball_outside((0.5, 0.5, 0.5), 0.3)


@pytest.fixture(scope="module")
def small2d():
    g = cg.make_geometry(CIRCLE, 16, 2)
    en, rp, col, val, st = oracle.build(g, 2)
    return g, en, rp, col, val, 2


@pytest.fixture(scope="module")
def small3d():
    g = cg.make_geometry(SPHERE, 8, 4)
    en, rp, col, val, st = oracle.build(g, 3)
    return g, en, rp, col, val, 3


def test_apply_adjoint_transpose_identity(small2d):
    """<lbar, L(Phi)> = <L^T lbar, Phi> (L is linear in Phi; Sec. 2.2)."""
    g, en, rp, col, val, R = small2d
    rng = np.random.default_rng(1)
    phi = rng.standard_normal(en.n_phi)
    lbar = rng.standard_normal(en.n_vol)
    _, L = oracle.apply(g, en, rp, col, val, phi)
    phi_bar, val_bar, kappa_bar = oracle.apply_adjoint(g, en, rp, col, val, phi, lbar)
    assert abs(np.dot(lbar, L) - np.dot(phi_bar, phi)) <= 1e-12 * np.abs(lbar).dot(np.abs(L))
    # the apply is bilinear in (val, Phi): <val_bar, val> = <lbar, L> as well
    assert abs(np.dot(val_bar, val) - np.dot(lbar, L)) <= 1e-12 * np.abs(lbar).dot(np.abs(L))


def test_apply_adjoint_kappa_by_finite_differences(small2d):
    g, en, rp, col, val, R = small2d
    rng = np.random.default_rng(2)
    phi = rng.standard_normal(en.n_phi)
    lbar = rng.standard_normal(en.n_vol)
    _, _, kappa_bar = oracle.apply_adjoint(g, en, rp, col, val, phi, lbar)
    for v in (3, 100, int(en.vol_of_cell[g.eb_cell[2]])):
        gg = copy.deepcopy(g)
        c = int(en.vol_cell[v])
        k0 = gg.vol_mom[c, 0]
        step = 1e-6 * k0
        vals = []
        for sgn in (1, -1):
            gg.vol_mom[c, 0] = k0 + sgn * step
            vals.append(np.dot(lbar, oracle.apply(gg, en, rp, col, val, phi)[1]))
        fd = (vals[0] - vals[1]) / (2 * step)
        assert abs(fd - kappa_bar[v]) <= 1e-7 * abs(kappa_bar[v])


def _fd_check(g, en, R, vb, G, items, rel_step=1e-4, tol=1e-6, faces=None):
    """Richardson-extrapolated central differences of sum(vb * val) over `faces`."""
    fl = range(en.n_face) if faces is None else faces
    base_en, rp0, col0, val0, _ = oracle.build(g, R, en=en, faces=fl)
    rp_full = np.zeros(en.n_face + 1, np.int64)
    rp_full[1:] = np.cumsum([len(oracle.neighbours(en, f, R)) for f in range(en.n_face)]) if faces is not None else 0
    vsel = (np.concatenate([vb[rp_full[f]:rp_full[f + 1]] for f in fl]) if faces is not None else vb)
    for kind, ix in items:
        gg = copy.deepcopy(g)
        if kind == "face":
            d, f, q = ix
            arr, key, ad = gg.face_mom[d], (f, q), G["face_mom"][d][f, q]
        else:
            arr = {"vol": gg.vol_mom, "eb": gg.eb_mom, "ebn": gg.eb_nmom}[kind]
            key = ix
            ad = {"vol": G["vol_mom"], "eb": G["eb_mom"], "ebn": G["eb_nmom"]}[kind][ix]
        b = arr[key]
        step = rel_step * max(abs(b), 1e-2)

        def central(hh):
            ls = []
            for sgn in (1, -1):
                arr[key] = b + sgn * hh
                e2 = oracle.enumerate_geometry(gg)
                _, rp2, col2, val2, _ = oracle.build(gg, R, en=e2, faces=fl)
                assert np.array_equal(col2, col0)
                ls.append(np.dot(vsel, val2))
            arr[key] = b
            return (ls[0] - ls[1]) / (2 * hh)

        fd = (4 * central(step / 2) - central(step)) / 3      # Richardson: O(step^4)
        scale = max(abs(ad), 1e-3 * np.abs(vb).max())
        assert abs(fd - ad) <= tol * scale, (kind, ix, fd, ad)


def test_stencil_gradients_by_finite_differences_2d(small2d):
    """d(sum val_bar * s)/d(moments): volume, EB, EB-normal and grid-face moments."""
    g, en, rp, col, val, R = small2d
    vb = np.random.default_rng(0).standard_normal(len(val))
    G = oracle.stencils_backward(g, en, R, rp, vb)
    cutc = int(g.eb_cell[3])
    items = [("vol", (cutc, 0)), ("vol", (cutc, 4)), ("vol", (int(en.vol_cell[5]), 2)), ("eb", (3, 1)),
             ("eb", (3, 0)), ("ebn", (3, 0, 1)), ("ebn", (3, 1, 0)), ("face", (0, int(en.face_lin[10]), 1))]
    _fd_check(g, en, R, vb, G, items)


def test_stencil_gradients_by_finite_differences_3d(small3d):
    """Same in 3D at fourth order, restricted to the faces around one cut cell (the
    EB face's x0 is the cut volume's centroid, so its volume moments enter every row)."""
    g, en, rp, col, val, R = small3d
    e = 5
    owner = int(en.vol_of_cell[g.eb_cell[e]])
    faces = [f for f in range(en.n_face) if owner in (en.face_lo[f], en.face_hi[f])]
    vb = np.zeros(len(val))
    rng = np.random.default_rng(3)
    for f in faces:
        vb[rp[f]:rp[f + 1]] = rng.standard_normal(rp[f + 1] - rp[f])
    G = oracle.stencils_backward(g, en, R, rp, vb, faces=faces)
    c = int(g.eb_cell[e])
    items = [("vol", (c, 0)), ("vol", (c, 1)), ("vol", (c, 7)), ("eb", (e, 0)), ("eb", (e, 12)),
             ("ebn", (e, 2, 3)), ("vol", (int(en.vol_cell[en.face_hi[faces[0]]]) if en.face_hi[faces[0]] >= 0 else c, 5))]
    _fd_check(g, en, R, vb, G, items, faces=faces)


def test_weight_gradient_is_scale_invariant(small2d):
    """s = W (A^T W)^+ F is unchanged when all weights of a face are scaled together, so
    sum_i W_i dl/dW_i = 0 face by face."""
    g, en, rp, col, val, R = small2d
    vb = np.random.default_rng(4).standard_normal(len(val))
    G = oracle.stencils_backward(g, en, R, rp, vb)
    for f in range(0, en.n_face, 7):
        A, W, F, idx = oracle.face_system(g, en, f, R)
        wb = G["weight"][rp[f]:rp[f + 1]]
        assert abs(np.dot(W, wb)) <= 1e-9 * np.abs(W).dot(np.abs(wb))
