"""Pins for the input generator (host quadrature of level-set cut cells).

The geometry is an input, not the method, but the oracle's convergence and
closed-form pins rely on moments accurate to rounding, so they are pinned here against
the paper's printed smallest volume fractions, closed forms and an independent
polygon computation.
"""

import math
import os

import numpy as np
import pytest

import cutgeom as cg

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _rows(name):
    out = []
    for line in open(os.path.join(GOLD, name)):
        if line.strip() and not line.startswith("#"):
            out.append(line.split())
    return out


@pytest.mark.parametrize("row", _rows("smallest_kappa_circle.txt"), ids=lambda r: "-".join(r[:4]))
def test_smallest_volume_fraction_matches_paper(row):
    """Sec. 3.4.1, table of smallest volume fractions: two printed digits."""
    x0, y0, r, N, k = row
    g = cg.make_geometry(cg.ball_outside((float(x0), float(y0)), float(r)), int(N), 2)
    kmin = g.kappa[g.state == 2].min()
    assert float("%.1e" % kmin) == float(k)


def test_disk_closed_forms():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5), 0.25), 64, 4)
    assert abs(g.kappa.sum() * g.h**2 - (1 - math.pi / 16)) < 1e-14
    assert abs(g.eb_mom[:, 0].sum() * g.h - 2 * math.pi * 0.25) < 1e-13
    # EB normal (out of the fluid = into the disk) integrates to zero
    assert np.abs(g.eb_nmom[:, :, 0].sum(axis=0)).max() < 1e-13


def test_star_area():
    g = cg.make_geometry(cg.star2_outside((0.5, 0.5), 0.25, 0.05, 6), 128, 4)
    exact = 1 - (math.pi * 0.25**2 + math.pi * 0.05**2 / 2)
    assert abs(g.kappa.sum() * g.h**2 - exact) < 1e-13


def test_sphere_closed_forms():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 32, 4)
    assert abs(g.kappa.sum() * g.h**3 - (1 - 4 / 3 * math.pi * 0.027)) < 1e-14
    assert abs(g.eb_mom[:, 0].sum() * g.h**2 - 4 * math.pi * 0.09) < 1e-13
    # second moment of the sphere surface about its centre: int |x-c|^2 dA = r^2 * area
    ci = np.array(np.unravel_index(g.eb_cell, g.n, order="F")).T
    c = (ci + 0.5) * g.h - 0.5
    mono = cg.monomials(3, 4)
    e = {p: k for k, p in enumerate(mono)}
    tot = 0.0
    for d in range(3):
        p1 = tuple(1 if i == d else 0 for i in range(3))
        p2 = tuple(2 if i == d else 0 for i in range(3))
        # (x_d - c0_d)^2 = (h xi + c_d)^2
        tot += np.sum(g.h**2 * g.eb_mom[:, e[p2]] + 2 * g.h * c[:, d] * g.eb_mom[:, e[p1]] + c[:, d] ** 2 * g.eb_mom[:, 0])
    assert abs(tot * g.h**2 - 0.09 * 4 * math.pi * 0.09) < 1e-13


def test_full_cell_moments_closed_form():
    g = cg.make_geometry(cg.ball_outside((0.5, 0.5, 0.5), 0.3), 16, 4)
    full = np.nonzero(g.state == 1)[0][0]
    for k, p in enumerate(cg.monomials(3, 4)):
        exact = np.prod([0.0 if q % 2 else 0.5**q / (q + 1) for q in p])
        assert g.vol_mom[full, k] == exact


@pytest.mark.parametrize("shape,n", [
    (cg.ball_outside((0.5, 0.5), 0.25), 32),
    (cg.ball_outside((0.5, 0.5, 0.5), 0.3), 16),
    (cg.sh_body_outside((0.5, 0.5, 0.5), 0.3, 0.01 * np.random.default_rng(4).standard_normal(16)), 16),
])
def test_divergence_identities(shape, n):
    """Per cut cell, int_dV n_d = 0 and int_dV xi_d n_d = kappa (divergence theorem)."""
    g = cg.make_geometry(shape, n, 4)
    D = g.D
    for e, c in enumerate(g.eb_cell):
        i = np.unravel_index(int(c), g.n, order="F")
        for d in range(D):
            m = g.face_dims(d)
            lo = list(i)
            hi = list(i)
            hi[d] += 1
            flo = np.ravel_multi_index(tuple(lo), m, order="F")
            fhi = np.ravel_multi_index(tuple(hi), m, order="F")
            a_lo, a_hi = g.face_mom[d][flo, 0], g.face_mom[d][fhi, 0]
            assert abs(a_hi - a_lo + g.eb_nmom[e, d, 0]) < 1e-13
            assert abs(0.5 * a_hi + 0.5 * a_lo + g.eb_nmom[e, d, 1 + d] - g.kappa[c]) < 1e-13


def _clip_polygon(poly, nrm, off):
    """Sutherland-Hodgman clip of a polygon to {n.x >= off}."""
    out = []
    for k in range(len(poly)):
        a, b = poly[k], poly[(k + 1) % len(poly)]
        fa, fb = nrm @ a - off, nrm @ b - off
        if fa >= 0:
            out.append(a)
        if (fa >= 0) != (fb >= 0):
            t = fa / (fa - fb)
            out.append(a + t * (b - a))
    return out


def test_planar_cut_matches_polygon_moments():
    """Half-plane cut: moments of the clipped polygons by Green's theorem on straight
    edges (exact Gauss-Legendre), independent of the level-set quadrature."""
    nrm = np.array([0.6, 0.8])
    off = 0.5123
    g = cg.make_geometry(cg.halfspace(nrm, off), 16, 4)
    xg, wg = np.polynomial.legendre.leggauss(8)
    mono = cg.monomials(2, 4)
    for c in np.nonzero(g.state == 2)[0]:
        i = np.array(np.unravel_index(int(c), g.n, order="F"), float)
        lo, ctr = i * g.h, (i + 0.5) * g.h
        sq = [np.array(v) for v in ((lo[0], lo[1]), (lo[0] + g.h, lo[1]), (lo[0] + g.h, lo[1] + g.h), (lo[0], lo[1] + g.h))]
        poly = _clip_polygon(sq, nrm, off)
        for k, (p, q) in enumerate(mono):
            # int_P xi^p eta^q dA = closed integral of xi^(p+1) eta^q / (p+1) d(eta)
            tot = 0.0
            for j in range(len(poly)):
                a, b = (poly[j] - ctr) / g.h, (poly[(j + 1) % len(poly)] - ctr) / g.h
                pts = 0.5 * (a + b)[None, :] + 0.5 * (b - a)[None, :] * xg[:, None]
                tot += np.sum(wg * 0.5 * pts[:, 0] ** (p + 1) * pts[:, 1] ** q / (p + 1)) * (b[1] - a[1])
            assert abs(g.vol_mom[c, k] - tot) < 1e-14, (c, p, q)
