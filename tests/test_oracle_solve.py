"""Pins for the oracle's Poisson solve (Sec. 3.2).

For a polynomial of degree <= Q every stencil is exact (Sec. 2.3: A^T s = F holds for
all monomials of degree <= Q), so with Phi holding the polynomial's exact averages the
divergence theorem gives L(Phi) = (exact integral of its Laplacian) / |V_v| in every
volume.  Solving L([x | Phi_bc]) = that right-hand side must then return the exact
volume averages: a wrong incidence sign, a dropped boundary term, a wrong volume scale or
a transposed operand each breaks it.  The solve is also pinned against the closed-form
Dirichlet problem with a constant Laplacian."""

import numpy as np
import pytest

import cutgeom as cg
import oracle

CIRCLE = cg.ball_outside((0.5, 0.5), 0.25)
SPHERE_IN = cg.ball_inside((0.5, 0.5, 0.5), 0.45)


def exact_phi_and_rhs(g, en, field):
    """Phi of the exact averages and the exact average Laplacian per volume."""
    I = g.integrate(field)
    hD, hD1 = g.h**g.D, g.h ** (g.D - 1)
    vol = en.vol_cell
    box = np.array([I["face_int"][d][f] / (g.face_mom[d][f, 0] * hD1) for d, f in zip(en.box_dir, en.box_face)])
    phi = np.concatenate([I["vol_int"][vol] / (g.kappa[vol] * hD), I["eb_int"] / (g.eb_mom[:, 0] * hD1), box])
    rhs = I["vol_lap"][vol] / (g.kappa[vol] * hD)
    return phi, rhs


@pytest.mark.parametrize("D,Q,R,N", [(2, 4, 3, 16), (2, 2, 2, 16), (3, 2, 2, 8)])
def test_solve_returns_exact_averages_of_polynomials(D, Q, R, N):
    shape = CIRCLE if D == 2 else SPHERE_IN
    g = cg.make_geometry(shape, N, Q)
    en, rp, col, val, status = oracle.build(g, R)
    assert np.all(status == oracle.STATUS_OK)
    field = cg.random_polynomial(D, Q, np.random.default_rng(11), scale=0.5)
    phi, rhs = exact_phi_and_rhs(g, en, field)
    x = oracle.solve(g, en, rp, col, val, phi, rhs)
    assert np.abs(x - phi[: en.n_vol]).max() <= 1e-9 * np.abs(phi).max()


def test_solve_with_constant_laplacian_matches_closed_form():
    """Inside the sphere of radius r: u = (|x - c|^2 - r^2) / 6 has Laplacian 1 and
    vanishes on the sphere; with u on the boundary the solve returns its averages."""
    g = cg.make_geometry(SPHERE_IN, 8, 2)
    en, rp, col, val, status = oracle.build(g, 2)
    # (|x-c|^2 - r^2)/6 as a polynomial about c: monomials x^2, y^2, z^2 and the constant
    mono = np.array([[0, 0, 0], [2, 0, 0], [0, 2, 0], [0, 0, 2]], float)
    amp = np.array([-0.45**2 / 6, 1 / 6, 1 / 6, 1 / 6])
    field = cg.PolyField(amp, mono, np.array([0.5, 0.5, 0.5]))
    phi, rhs = exact_phi_and_rhs(g, en, field)
    assert np.allclose(rhs, 1.0, atol=1e-13)
    assert np.abs(phi[en.n_vol: en.n_vol + en.n_eb]).max() < 1e-13       # u = 0 on the sphere
    x = oracle.solve(g, en, rp, col, val, phi, rhs)
    assert np.abs(x - phi[: en.n_vol]).max() <= 1e-11
    assert np.all(x < 0)                                                 # u < 0 inside


def test_operator_matrix_matches_apply():
    """The assembled matrix and the face-by-face apply are the same map."""
    g = cg.make_geometry(CIRCLE, 16, 2)
    en, rp, col, val, status = oracle.build(g, 2)
    phi = np.random.default_rng(3).standard_normal(en.n_phi)
    _, L = oracle.apply(g, en, rp, col, val, phi)
    Lm = oracle.operator_matrix(g, en, rp, col, val) @ phi
    assert np.abs(L - Lm).max() <= 1e-12 * np.abs(L).max()
