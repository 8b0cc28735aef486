"""Oracle Poisson solve with the flux-divergence operator.

Test infrastructure only (see the package docstring).

Sec. 3.2 solves the discrete system L(Phi) = f for the volume values of Phi, the EB and
box entries of Phi holding Dirichlet data.  Here L is assembled as a sparse matrix,
straight from its definition (Sec. 2.2, eq. 'laplacian over V'):

    L = diag(1 / |V_v|) . Sigma . S

with S the n_face x n_phi matrix of the stencils (flux_f = s_f^T Phi), Sigma the
n_vol x n_face signed incidence (+1 where the face's reference normal points out of the
volume), and the volume system  L[:, vols] x = f - L[:, rest] Phi_rest  is solved by a
sparse LU factorisation (SuperLU through scipy), the library step.
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp
import scipy.sparse.linalg as spl


def operator_matrix(geom, en, row_ptr, col, val):
    """L as a sparse n_vol x n_phi matrix (Sec. 2.2, eq. 'laplacian over V')."""
    S = sp.csr_matrix((val, col, row_ptr), shape=(en.n_face, en.n_phi))
    rows, cols, sgn = [], [], []
    for f in range(en.n_face):
        if en.face_lo[f] >= 0:           # the face is the high face of this volume
            rows.append(en.face_lo[f])
            cols.append(f)
            sgn.append(1.0)
        if en.face_hi[f] >= 0:           # the face is the low face of this volume
            rows.append(en.face_hi[f])
            cols.append(f)
            sgn.append(-1.0)
    Sigma = sp.csr_matrix((sgn, (rows, cols)), shape=(en.n_vol, en.n_face))
    kappa = geom.vol_mom[en.vol_cell, 0]
    return (sp.diags(1.0 / (kappa * en.h**en.D)) @ Sigma @ S).tocsr()


def solve(geom, en, row_ptr, col, val, phi_bc, rhs):
    """Volume values x with L([x | Phi_bc]) = rhs (Sec. 3.2), by a sparse direct solve.
    phi_bc: [n_phi], its volume entries ignored; rhs: [n_vol]."""
    L = operator_matrix(geom, en, row_ptr, col, val)
    nv = en.n_vol
    b = rhs - L[:, nv:] @ phi_bc[nv:]
    return spl.spsolve(L[:, :nv].tocsc(), b)
