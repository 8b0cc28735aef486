"""Pins for the oracle's neighbour rule (Sec. 2.4, readings R1 and R2) against rows
derived by hand on drawn masks (tests/golden/neighbours_2d.txt): an L-shaped obstacle
where path distance and L1 distance differ, a box corner, a cut cell whose EB face is
reached only through a neighbour, the EB face's own rows, and a one-cell channel that
opens into a room."""

import os

import numpy as np
import pytest

import cutgeom as cg
import oracle
from oracle import stencils as S

GOLD = os.path.join(os.path.dirname(__file__), "golden", "neighbours_2d.txt")


def _read():
    masks, faces = {}, []
    lines = [ln.rstrip("\n") for ln in open(GOLD)]
    k = 0
    while k < len(lines):
        ln = lines[k]
        if ln.startswith("mask "):
            name = ln.split()[1]
            rows = lines[k + 1:k + 9]
            masks[name] = rows
            k += 9
            continue
        if ln.startswith("face "):
            head, tail = ln.split(":")
            _, m, kind, d, i, j, R = head.split()
            faces.append((m, kind, int(d), int(i), int(j), int(R), [int(x) for x in tail.split()]))
        k += 1
    return masks, faces


def _mask_geometry(rows):
    """An 8 x 8 geometry from the drawn mask: full cells, covered cells and cut cells
    carrying an EB face; a grid face has area 1 between two volumes and 0 otherwise,
    a box face area 1 next to a volume."""
    n = 8
    g = cg.make_geometry(cg.halfspace([0.0, 1.0], -1.0), n, 2)   # all fluid, no EB faces
    kind = np.zeros(n * n, dtype=np.int64)    # 0 covered, 1 volume, 2 cut
    for r, text in enumerate(rows):
        j = n - 1 - r
        for i, ch in enumerate(text):
            kind[i + n * j] = {"#": 0, ".": 1, "c": 2}[ch]
    full = g.vol_mom[0].copy()
    g.vol_mom[:] = 0
    g.vol_mom[kind > 0] = full
    g.vol_mom[kind == 2, 0] = 0.5
    for d in range(2):
        m = g.face_dims(d)
        for f in range(len(g.face_mom[d])):
            jj = list(np.unravel_index(f, m, order="F"))
            lo, hi = list(jj), list(jj)
            lo[d] -= 1
            sides = [c for c in (lo, hi) if 0 <= c[d] < n]
            vols = [kind[c[0] + n * c[1]] > 0 for c in sides]
            g.face_mom[d][f] = 0
            g.face_mom[d][f, 0] = 1.0 if all(vols) else 0.0
    cut = np.flatnonzero(kind == 2).astype(np.int32)
    g.eb_cell = cut
    g.eb_mom = np.tile(g.vol_mom[0], (len(cut), 1))
    g.eb_nmom = np.zeros((len(cut), 2, g.M1))
    g.state = np.where(kind == 0, 0, np.where(kind == 1, 1, 2)).astype(np.int8)
    return g


MASKS, FACES = _read()


def test_fixture_is_complete():
    assert set(MASKS) == {"A", "B"} and len(FACES) == 5
    for rows in MASKS.values():
        assert len(rows) == 8 and all(len(r) == 8 for r in rows)


@pytest.mark.parametrize("face", FACES, ids=[f"{f[0]}-{f[1]}-{f[2]}-{f[3]}-{f[4]}" for f in FACES])
def test_neighbours_match_hand_derived_rows(face):
    m, kind, d, i, j, R, expected = face
    g = _mask_geometry(MASKS[m])
    en = oracle.enumerate_geometry(g)
    if kind == "eb":
        e = int(np.flatnonzero(en.eb_cell == i + 8 * j)[0])
        f = int(np.flatnonzero((en.face_kind == S.KIND_EB) & (en.face_lin == e))[0])
    else:
        lin = np.ravel_multi_index((i, j), g.face_dims(d), order="F")
        f = int(np.flatnonzero((en.face_kind != S.KIND_EB) & (en.face_dir == d) & (en.face_lin == lin))[0])
        assert en.face_kind[f] == (S.KIND_BOX if kind == "box" else S.KIND_GRID)
    got = oracle.neighbours(en, f, R)
    assert list(got) == expected


@pytest.mark.parametrize("case", ["maskA", "maskB", "circle16", "star32", "sphere8", "sphere8_r2"])
def test_all_face_rows_at_once_match_face_by_face(case):
    """neighbours_all (sparse reachability, used for the full-size bit-exact checks) gives
    exactly the rows of neighbours() on every face."""
    if case.startswith("mask"):
        g, R = _mask_geometry(MASKS[case[-1]]), 2
    else:
        shape, n, Q, R = {"circle16": (cg.ball_outside((0.5, 0.5), 0.25), 16, 2, 2),
                          "star32": (cg.star2_outside((0.5, 0.5), 0.25, 0.05, 6), 32, 4, 3),
                          "sphere8": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 8, 4, 3),
                          "sphere8_r2": (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 8, 2, 2)}[case]
        g = cg.make_geometry(shape, n, Q)
    en = oracle.enumerate_geometry(g)
    rp, col = oracle.neighbours_all(en, R)
    for f in range(en.n_face):
        assert list(col[rp[f]:rp[f + 1]]) == list(oracle.neighbours(en, f, R)), f
