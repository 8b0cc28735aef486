"""Pins for the oracle's Neumann embedded-boundary rows (Sec. 2.2.1, eq. 'Neu moment eq
for cp'; case 3 of Sec. 3.4: Neumann on the circle, Dirichlet on the square).

* Exactness: for a polynomial of degree <= Q, with each Neumann EB entry of Phi holding
  the average normal derivative (from an independent quadrature), every face flux s^T Phi
  equals the exact flux and the solve returns the exact volume averages.  A wrong
  normal-row formula, a missing h on the Neumann values or a wrong EB-face flux breaks it.
* The paper's spectrum of the 64 x 64 Neumann operator: lambda_max = -38 (the smallest
  eigenvalue in magnitude is a property of the continuous problem, so the 32 x 32 grid
  already shows it), all eigenvalues in the left half plane.
* The paper's Neumann solution-error table at N = 32 and 64.
"""

import math
import os

import numpy as np
import pytest

import cutgeom as cg
import oracle
from oracle import stencils as S

GOLD = os.path.join(os.path.dirname(__file__), "golden")
CIRCLE = cg.ball_outside((0.5, 0.5), 0.25)
SPHERE = cg.ball_outside((0.5, 0.5, 0.5), 0.3)
NEU = "neumann"


def _paper():
    out = {}
    for line in open(os.path.join(GOLD, "circle_neumann_paper_numbers.txt")):
        if line.strip() and not line.startswith("#"):
            k, *v = line.split()
            out[k] = [float(x) if x != "-" else None for x in v]
    return out


PAPER = _paper()


def neumann_phi_and_rhs(g, en, I):
    """Phi with volume averages, the average normal derivative on EB faces and box-face
    averages; the average Laplacian per volume."""
    hD, hD1 = g.h**g.D, g.h ** (g.D - 1)
    vol = en.vol_cell
    box = np.array([I["face_int"][d][f] / (g.face_mom[d][f, 0] * hD1) for d, f in zip(en.box_dir, en.box_face)])
    phi = np.concatenate([I["vol_int"][vol] / (g.kappa[vol] * hD), I["eb_flux"] / (g.eb_mom[:, 0] * hD1), box])
    return phi, I["vol_lap"][vol] / (g.kappa[vol] * hD)


def _exact_flux(en, I):
    out = np.empty(en.n_face)
    grid = en.face_kind != S.KIND_EB
    for d in range(en.D):
        m = grid & (en.face_dir == d)
        out[m] = I["face_flux"][d][en.face_lin[m]]
    out[~grid] = I["eb_flux"][en.face_lin[~grid]]
    return out


@pytest.mark.parametrize("D,Q,R,N", [(2, 4, 3, 16), (2, 2, 2, 16), (3, 2, 2, 8), (3, 4, 3, 8)])
def test_neumann_fluxes_exact_for_polynomials(D, Q, R, N):
    g = cg.make_geometry(CIRCLE if D == 2 else SPHERE, N, Q)
    en, rp, col, val, st = oracle.build(g, R, eb_bc=NEU)
    assert np.all(st == oracle.STATUS_OK)
    I = g.integrate(cg.random_polynomial(D, Q, np.random.default_rng(21), scale=0.5))
    phi, _ = neumann_phi_and_rhs(g, en, I)
    flux, _ = oracle.apply(g, en, rp, col, val, phi)
    ref = _exact_flux(en, I)
    absterm = np.add.reduceat(np.abs(val) * np.abs(phi[col]), rp[:-1])
    assert np.all(np.abs(flux - ref) <= 1e-10 * (absterm + np.abs(ref)))
    # the EB faces' own stencils are their areas on their own entries
    eb = np.flatnonzero(en.face_kind == S.KIND_EB)
    assert np.all(np.diff(rp)[eb] == 1)
    assert np.array_equal(col[rp[eb]], en.n_vol + en.face_lin[eb])


def test_neumann_solve_exact_for_polynomials():
    g = cg.make_geometry(CIRCLE, 16, 4)
    en, rp, col, val, st = oracle.build(g, 3, eb_bc=NEU)
    I = g.integrate(cg.random_polynomial(2, 4, np.random.default_rng(22), scale=0.5))
    phi, rhs = neumann_phi_and_rhs(g, en, I)
    x = oracle.solve(g, en, rp, col, val, phi, rhs)
    assert np.abs(x - phi[: en.n_vol]).max() <= 1e-9 * np.abs(phi).max()


def test_neumann_differs_from_dirichlet_only_near_the_boundary():
    """Faces whose rows hold no EB entry get the same stencil under either condition."""
    g = cg.make_geometry(CIRCLE, 16, 4)
    en, rp, col, val, _ = oracle.build(g, 3)
    en2, rp2, col2, val2, _ = oracle.build(g, 3, en=en, eb_bc=NEU)
    for f in range(en.n_face):
        a, b = rp[f], rp[f + 1]
        has_eb = np.any((col[a:b] >= en.n_vol) & (col[a:b] < en.n_vol + en.n_eb))
        if not has_eb and en.face_kind[f] != S.KIND_EB:
            assert np.array_equal(col[a:b], col2[rp2[f]:rp2[f + 1]])
            assert np.array_equal(val[a:b], val2[rp2[f]:rp2[f + 1]])


def test_neumann_spectrum_matches_paper():
    g = cg.make_geometry(CIRCLE, 32, 4)
    en, rp, col, val, st = oracle.build(g, 3, eb_bc=NEU)
    A = oracle.operator_matrix(g, en, rp, col, val)[:, : en.n_vol].toarray()
    ev = np.linalg.eigvals(A)
    lam_max = ev.real.max()
    assert lam_max < 0
    assert abs(lam_max - PAPER["lambda_max_64"][0]) < 3.0


def _neumann_errors(N):
    g = cg.make_geometry(CIRCLE, N, 4)
    en, rp, col, val, st = oracle.build(g, 3, eb_bc=NEU)
    tp = 2 * math.pi
    I = g.integrate(cg.trig_product((tp, tp), (-tp * math.sqrt(2) / 2, -tp * math.sqrt(3) / 2)))
    phi, rhs = neumann_phi_and_rhs(g, en, I)
    x = oracle.solve(g, en, rp, col, val, phi, rhs)
    e = x - phi[: en.n_vol]
    V = g.kappa[en.vol_cell] * g.h**2
    return dict(soln_Linf=np.abs(e).max(), soln_L1=np.sum(np.abs(e) * V) / V.sum())


@pytest.mark.slow
def test_neumann_circle_solution_errors():
    """Case 3 of Sec. 3.4 at N = 32 and 64: fourth order, errors within a factor 2 of the
    paper's table (volume-weighted mean for L1)."""
    e = {N: _neumann_errors(N) for N in (32, 64)}
    for k in ("soln_Linf", "soln_L1"):
        assert math.log2(e[32][k] / e[64][k]) > 3.6, k
        for i, N in enumerate((32, 64)):
            assert 0.5 < e[N][k] / PAPER[k][i] < 2.0, (k, N, e[N][k], PAPER[k][i])
