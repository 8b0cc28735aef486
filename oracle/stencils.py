"""Oracle: flux stencils and the flux-divergence operator, straight from the paper.

Test infrastructure only (see the package docstring).

Paper references are to arXiv:1411.4283 by section, equation label or table:
  Sec. 2.1   spatial notation: volumes, grid-aligned faces, boundary faces, moments
  Sec. 2.2   flux approximation; Sec. 2.2.1 the polynomial interpolant, the system
             A c = Phi (eq. 'def of A', 'def of phi vec'), the stencil
             s = W (A^T W)^+ F (eq. 'stencil equation solution')
  Sec. 2.4   neighbours (path radius R_n) and the weights W_ii
  Sec. 3.3   face flux s_f^T Phi and the divergence over the faces of a volume

Scaled quantities (the input moments are scaled, see ``cutgeom``): with
xi = (x - x0)/h, the scaled rows A~ and flux vector F~ give the scaled stencil
s~ = W (A~^T W)^+ F~, and the physical stencil is s = h^(D-2) s~, because scaling the
columns of A and the entries of F by h^|p| leaves both A^T s = F and the
minimised norm ||W^-1 s|| unchanged.

Arithmetic.  The inputs (moments) are FP64 numbers, taken as exact.  Everything the
stencil is computed from them with -- the offsets (x_i - x0)/h, the weights, the
re-centred rows and the factorisation -- is carried in x87 extended precision
(numpy.longdouble, unit roundoff 5.4e-20) and rounded to FP64 once at the end: the
oracle's own error on a face is then about cond * 1e-19, far below the 1e-11 at which
stencils are compared, for every system of condition number up to ~1e7.  The offsets are
formed in units of h from cell and lattice indices, so for grid and box faces they are the
exact half-integers the geometry defines, whatever h is.

Readings of points the paper leaves open are tagged R1..R16 (listed in the design
notes); they are the same for the HIP library.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from functools import lru_cache
from math import comb

import numpy as np

import cutgeom

STATUS_OK = 0
STATUS_INSUFFICIENT_ROWS = 1
STATUS_RANK_DEFICIENT = 2
STATUS_NONFINITE = 3

# A face is flagged rank deficient when the triangular factor of the Householder QR of
# its column-equilibrated weighted matrix has min|R_kk| <= RANK_TOL * max|R_kk| (reading
# R8: Sec. 2.2.1 assumes a full-rank system; at this ratio an FP64 system no longer fixes
# its stencil to better than about 1e-4).
RANK_TOL = 1e-12

LD = np.longdouble

KIND_GRID, KIND_BOX, KIND_EB = 0, 1, 2


@lru_cache(maxsize=None)
def _mono(D, Q):
    return tuple(cutgeom.monomials(D, Q))


@lru_cache(maxsize=None)
def _shift_terms(D, Q):
    """Terms of the binomial re-centring of moments (multi-index binomial theorem):
    m^p(x0) = sum_{q <= p} C(p,q) (c - x0)^(p-q) m^q(c).
    Returns (coef[T], exponent p-q [T, D], index of q [T], 0/1 matrix T x M mapping
    each term to its p)."""
    mono = _mono(D, Q)
    coef, ex, qi, pi = [], [], [], []
    for a, p in enumerate(mono):
        for b, q in enumerate(mono):
            if all(qq <= pp for pp, qq in zip(p, q)):
                coef.append(float(np.prod([comb(pp, qq) for pp, qq in zip(p, q)])))
                ex.append([pp - qq for pp, qq in zip(p, q)])
                qi.append(b)
                pi.append(a)
    P = np.zeros((len(pi), len(mono)))
    P[np.arange(len(pi)), pi] = 1.0
    return np.array(coef), np.array(ex, dtype=np.int64), np.array(qi), P


# ---------------------------------------------------------------------------------
# Sec. 2.1: volumes, boundary faces and flux faces


@dataclass
class Enumeration:
    D: int
    n: tuple
    h: float
    Q: int
    vol_cell: np.ndarray      # cell of each volume, ascending
    vol_of_cell: np.ndarray   # dense map cell -> volume index (-1 if covered)
    eb_cell: np.ndarray       # cell of each EB face (input order, ascending)
    eb_of_cell: np.ndarray    # dense map cell -> EB index (-1)
    box_dir: np.ndarray       # box faces in Phi order: direction, side (0 low, 1 high),
    box_side: np.ndarray      #   face-lattice index and adjacent cell
    box_face: np.ndarray
    box_cell: np.ndarray
    face_kind: np.ndarray     # flux faces: 0 grid interior, 1 box, 2 EB
    face_dir: np.ndarray      # direction d (grid/box), -1 (EB)
    face_lin: np.ndarray      # face-lattice index (grid/box) or EB index
    face_lo: np.ndarray       # volume on the low side (-1 for a box face at x_d = 0);
                              # for an EB face: its owner
    face_hi: np.ndarray       # volume on the high side (-1 at x_d = 1 and for EB faces)
    vol_adj: list = field(repr=False, default=None)    # face-neighbour volumes of each volume
    vol_box: list = field(repr=False, default=None)    # box faces (Phi-order index) of each volume
    row_mom: np.ndarray = field(repr=False, default=None)  # moments of each Phi row about its centre
    row_ctr: np.ndarray = field(repr=False, default=None)  # centre x_i of each Phi row
    row_ctr_h: np.ndarray = field(repr=False, default=None)  # the same in units of h (exact
                                                              # half-integers)

    @property
    def n_vol(self):
        return len(self.vol_cell)

    @property
    def n_eb(self):
        return len(self.eb_cell)

    @property
    def n_box(self):
        return len(self.box_dir)

    @property
    def n_phi(self):
        return self.n_vol + self.n_eb + self.n_box

    @property
    def n_face(self):
        return len(self.face_kind)


def _strides(n):
    s = [1]
    for v in n[:-1]:
        s.append(s[-1] * v)
    return s


def _face_lattice(n, d):
    m = list(n)
    m[d] += 1
    return tuple(m)


def enumerate_geometry(geom) -> Enumeration:
    """Volumes, boundary faces and flux faces of a single-valued cut-cell grid (Sec. 2.1).

    Phi (eq. 'def of phi vec') is ordered [volumes | EB faces | box faces]: volumes by
    cell index; EB faces in input order; box faces by (direction, low/high side, index
    of the adjacent cell).  Flux faces (one stencil each) are the grid-aligned faces of
    area fraction > 0 in order (direction, face-lattice index), box faces included,
    followed by the EB faces.
    """
    D, n, Q, h = geom.D, tuple(geom.n), geom.Q, geom.h
    ncell = int(np.prod(n))
    cells = np.arange(ncell)
    ci = np.array(np.unravel_index(cells, n, order="F"))          # [D, ncell]
    kappa = geom.vol_mom[:, 0]
    vol_cell = np.nonzero(kappa > 0)[0]
    vol_of_cell = -np.ones(ncell, dtype=np.int64)
    vol_of_cell[vol_cell] = np.arange(len(vol_cell))
    eb_cell = np.asarray(geom.eb_cell, dtype=np.int64)
    eb_of_cell = -np.ones(ncell, dtype=np.int64)
    eb_of_cell[eb_cell] = np.arange(len(eb_cell))

    bd, bs, bf, bc = [], [], [], []
    for d in range(D):
        m = _face_lattice(n, d)
        for side in (0, 1):
            sel = cells[ci[d] == (0 if side == 0 else n[d] - 1)]
            j = ci[:, sel].copy()
            j[d] += side
            f = np.ravel_multi_index(tuple(j), m, order="F")
            keep = geom.face_mom[d][f, 0] > 0
            bd.append(np.full(keep.sum(), d))
            bs.append(np.full(keep.sum(), side))
            bf.append(f[keep])
            bc.append(sel[keep])
    box_dir, box_side, box_face, box_cell = (np.concatenate(x).astype(np.int64) for x in (bd, bs, bf, bc))

    kind, fdir, flin, flo, fhi = [], [], [], [], []
    for d in range(D):
        m = _face_lattice(n, d)
        f = np.nonzero(geom.face_mom[d][:, 0] > 0)[0]
        j = np.array(np.unravel_index(f, m, order="F"))
        lo_ok = j[d] >= 1
        hi_ok = j[d] <= n[d] - 1
        jl = j.copy()
        jl[d] -= 1
        lo = np.where(lo_ok, vol_of_cell[np.ravel_multi_index(tuple(np.where(lo_ok, jl, 0)), n, order="F")], -1)
        jh = np.where(hi_ok, j, 0)
        hi = np.where(hi_ok, vol_of_cell[np.ravel_multi_index(tuple(jh), n, order="F")], -1)
        kind.append(np.where((lo >= 0) & (hi >= 0), KIND_GRID, KIND_BOX))
        fdir.append(np.full(len(f), d))
        flin.append(f)
        flo.append(lo)
        fhi.append(hi)
    ne = len(eb_cell)
    kind.append(np.full(ne, KIND_EB))
    fdir.append(np.full(ne, -1))
    flin.append(np.arange(ne))
    flo.append(vol_of_cell[eb_cell])
    fhi.append(np.full(ne, -1))
    cat = lambda x: np.concatenate(x).astype(np.int64)  # noqa: E731
    en = Enumeration(D, n, h, Q, vol_cell, vol_of_cell, eb_cell, eb_of_cell, box_dir, box_side,
                     box_face, box_cell, cat(kind), cat(fdir), cat(flin), cat(flo), cat(fhi))

    # volume graph: volumes joined by a grid-aligned face of positive area
    adj = [[] for _ in range(len(vol_cell))]
    for f in np.nonzero(en.face_kind == KIND_GRID)[0]:
        a, b = int(en.face_lo[f]), int(en.face_hi[f])
        adj[a].append(b)
        adj[b].append(a)
    en.vol_adj = adj
    vb = [[] for _ in range(len(vol_cell))]
    for b in range(len(box_dir)):
        vb[int(vol_of_cell[box_cell[b]])].append(b)
    en.vol_box = vb

    # each Phi row's moments about its own centre, as D-variate vectors, and the centre:
    # volumes use cell moments about the cell centre; EB faces their moments about the
    # cut cell's centre; box faces the transverse face moments about the face centre,
    # embedded with exponent 0 in the face's normal direction.
    mono = _mono(D, Q)
    M = len(mono)
    rm = np.zeros((en.n_phi, M))
    rc = np.zeros((en.n_phi, D))
    rm[: en.n_vol] = geom.vol_mom[vol_cell]
    rc[: en.n_vol] = ci[:, vol_cell].T + 0.5
    rm[en.n_vol: en.n_vol + ne] = geom.eb_mom
    rc[en.n_vol: en.n_vol + ne] = ci[:, eb_cell].T + 0.5
    monof = {q: k for k, q in enumerate(_mono(D - 1, Q))}
    o = en.n_vol + ne
    for d in range(D):
        embed = [(a, monof[tuple(p[e] for e in range(D) if e != d)]) for a, p in enumerate(mono) if p[d] == 0]
        sel = np.nonzero(box_dir == d)[0]
        for a, k in embed:
            rm[o + sel, a] = geom.face_mom[d][box_face[sel], k]
        j = np.array(np.unravel_index(box_face[sel], _face_lattice(n, d), order="F")).T.astype(np.float64)
        x = j + 0.5
        x[:, d] = j[:, d]
        rc[o + sel] = x
    en.row_mom = rm
    en.row_ctr_h = rc
    en.row_ctr = rc * h
    return en


# ---------------------------------------------------------------------------------
# Sec. 2.4: neighbours by path radius


def volumes_within(en: Enumeration, v0: int, R: int) -> set:
    """Volumes at path distance <= R from v0 through grid-aligned faces of positive area
    (Sec. 2.4, 'path radius'; reading R1)."""
    seen = {v0}
    frontier = [v0]
    for _ in range(R):
        nxt = []
        for v in frontier:
            for u in en.vol_adj[v]:
                if u not in seen:
                    seen.add(u)
                    nxt.append(u)
        frontier = nxt
    return seen


def neighbours(en: Enumeration, f: int, R: int) -> np.ndarray:
    """Phi indices of the rows of face f, ascending (Sec. 2.4): the volumes within path
    radius R of the face's adjacent volumes, then the boundary faces (EB and box faces)
    those volumes touch (readings R1, R2)."""
    adj = [int(v) for v in (en.face_lo[f], en.face_hi[f]) if v >= 0]
    S = set()
    for a in adj:
        S |= volumes_within(en, a, R)
    vols = sorted(S)
    ebs = sorted(int(en.eb_of_cell[en.vol_cell[v]]) for v in vols if en.eb_of_cell[en.vol_cell[v]] >= 0)
    boxes = sorted(b for v in vols for b in en.vol_box[v])
    idx = vols + [en.n_vol + e for e in ebs] + [en.n_vol + en.n_eb + b for b in boxes]
    return np.asarray(idx, dtype=np.int64)


def neighbours_all(en: Enumeration, R: int):
    """The rows of every flux face at once, as CSR (row_ptr, col), the same sets as
    neighbours() face by face (Sec. 2.4; readings R1, R2), from sparse matrices: with A the
    adjacency of volumes through grid faces of positive area, the volumes within path
    distance R of volume v are the nonzero pattern of row v of (I + A)^R; a face's volumes
    are the union over its adjacent volumes; its EB and box rows are those of the volumes
    in that union.  Columns ascending: volumes, EB faces, box faces."""
    import scipy.sparse as sp

    nv, nf = en.n_vol, en.n_face
    grid = en.face_kind == KIND_GRID
    lo, hi = en.face_lo[grid], en.face_hi[grid]
    A = sp.csr_matrix((np.ones(2 * len(lo)), (np.concatenate([lo, hi]), np.concatenate([hi, lo]))), shape=(nv, nv))
    step = (sp.identity(nv, format="csr") + A).tocsr()
    step.data[:] = 1.0
    reach = sp.identity(nv, format="csr")
    for _ in range(R):
        reach = (reach @ step).tocsr()
        reach.data[:] = 1.0
    has_lo, has_hi = en.face_lo >= 0, en.face_hi >= 0
    rows = np.concatenate([np.flatnonzero(has_lo), np.flatnonzero(has_hi)])
    cols = np.concatenate([en.face_lo[has_lo], en.face_hi[has_hi]])
    adj = sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(nf, nv))
    fv = (adj @ reach).tocsr()
    ve = sp.csr_matrix((np.ones(en.n_eb), (en.vol_of_cell[en.eb_cell], np.arange(en.n_eb))), shape=(nv, en.n_eb))
    vb = sp.csr_matrix((np.ones(en.n_box), (en.vol_of_cell[en.box_cell], np.arange(en.n_box))), shape=(nv, en.n_box))
    full = sp.hstack([fv, fv @ ve, fv @ vb], format="csr")
    full.sort_indices()
    return full.indptr.astype(np.int64), full.indices.astype(np.int64)


# ---------------------------------------------------------------------------------
# Sec. 2.2.1: rows of A, the weights and the flux vector


def face_centre_h(en: Enumeration, f: int, eb_x0: str = "centroid") -> np.ndarray:
    """x0 / h of face f (Sec. 2.4), in extended precision: the face centre for a
    grid-aligned face; for an EB face the centre of the cell it cuts, read as the
    centroid of the cut volume, c + (first moments / zeroth moment) (reading R3;
    ``eb_x0="cell"`` takes the Cartesian cell centre instead, the literal reading, which
    gives an operator with positive eigenvalues on the paper's circle)."""
    if en.face_kind[f] == KIND_EB:
        v = int(en.face_lo[f])
        c = en.row_ctr_h[v].astype(LD)
        if eb_x0 == "cell":
            return c
        m = en.row_mom[v].astype(LD)
        return c + m[1 : en.D + 1] / m[0]
    d = int(en.face_dir[f])
    j = np.array(np.unravel_index(int(en.face_lin[f]), _face_lattice(en.n, d), order="F"), dtype=LD)
    x = j + LD(0.5)
    x[d] = j[d]
    return x


def face_centre(en: Enumeration, f: int, eb_x0: str = "centroid") -> np.ndarray:
    """x0 of face f in physical coordinates (FP64), see face_centre_h."""
    return (face_centre_h(en, f, eb_x0) * LD(en.h)).astype(np.float64)


def recentre(mom: np.ndarray, delta: np.ndarray, D: int, Q: int) -> np.ndarray:
    """Moments about x0 from moments about c (multi-index binomial theorem):
    m^p(x0) = sum_{q <= p} C(p,q) delta^(p-q) m^q(c),  delta = (c - x0)/h, scaled.
    ``mom`` is [..., M], ``delta`` is [..., D]."""
    coef, ex, qi, P = _shift_terms(D, Q)
    # delta_d^k for k = 0..Q by repeated products, then the product over the directions
    pw = [np.ones_like(delta)]
    for _ in range(Q):
        pw.append(pw[-1] * delta)
    pw = np.stack(pw, axis=-1)                                    # [..., D, Q+1]
    powers = pw[..., 0, ex[:, 0]]
    for d in range(1, D):
        powers = powers * pw[..., d, ex[:, d]]                    # [..., T]
    # the terms come grouped by p (ascending), so each m^p(x0) is the sum of one run
    starts = np.searchsorted(np.argmax(P, axis=1), np.arange(P.shape[1]))
    return np.add.reduceat(coef * powers * mom[..., qi], starts, axis=-1)


def row_weights(dist_over_h: np.ndarray, wpow: float = 5.0) -> np.ndarray:
    """W_ii of Sec. 2.4: 1 if |x_i - x0|/h < 1/2, else (2 |x_i - x0|/h)^-5; `wpow`
    replaces the exponent 5 for weight studies (0: unweighted least squares)."""
    d = np.asarray(dist_over_h)
    if d.dtype != LD:
        d = d.astype(np.float64)
    one = d.dtype.type(1)
    return np.where(d < 0.5, one, (2 * np.maximum(d, d.dtype.type(0.5))) ** (-d.dtype.type(wpow)))


def flux_vector(geom, en: Enumeration, f: int, x0h: np.ndarray) -> np.ndarray:
    """Scaled flux vector F~_p = int_f grad(xi^p) . n dA_xi, xi = (x - x0)/h (Sec. 2.2).

    Grid/box face of direction d (reference normal +e_d, x0 the face centre, so the face
    lies on xi_d = 0): d/dxi_d xi^p = p_d xi^(p - e_d) vanishes on the face unless
    p_d = 1, so F~_p = face moment of exponent p - e_d.  EB face (normal out of the
    fluid): F~_p = sum_d p_d (EB normal moment of exponent p - e_d, component d) about
    x0 (the identity used in Sec. 2.3); the stored normal moments, taken about the cell
    centre, are re-centred to x0 (x0h = x0 / h, extended precision)."""
    D, Q = en.D, en.Q
    mono = _mono(D, Q)
    F = np.zeros(len(mono), dtype=LD)
    if en.face_kind[f] == KIND_EB:
        return eb_normal_flux(geom, en, int(en.face_lin[f]), x0h)
    d = int(en.face_dir[f])
    monof = {q: k for k, q in enumerate(_mono(D - 1, Q))}
    for a, p in enumerate(mono):
        if p[d] == 1:
            F[a] = geom.face_mom[d][en.face_lin[f], monof[tuple(p[k] for k in range(D) if k != d)]]
    return F


def eb_normal_flux(geom, en: Enumeration, e: int, x0h: np.ndarray) -> np.ndarray:
    """sum_d p_d (normal moment of exponent p - e_d, component d) of EB face e about x0,
    scaled: the flux of each monomial xi^p through the face (Sec. 2.3), and, divided by
    the face area, the Neumann row of eq. 'Neu moment eq for cp'.  The stored normal
    moments, taken about the cell centre, are re-centred to x0 by the binomial theorem
    (x0h = x0 / h; extended precision)."""
    D, Q = en.D, en.Q
    mono = _mono(D, Q)
    F = np.zeros(len(mono), dtype=LD)
    c = en.row_ctr_h[en.n_vol + e].astype(LD)
    nu = recentre(geom.eb_nmom[e].astype(LD), np.broadcast_to(c - x0h, (D, D)), D, Q - 1)   # [D, M1]
    mono1 = {q: k for k, q in enumerate(_mono(D, Q - 1))}
    for a, p in enumerate(mono):
        for d in range(D):
            if p[d] > 0:
                q = list(p)
                q[d] -= 1
                F[a] += p[d] * nu[d, mono1[tuple(q)]]
    return F


def face_system_ld(geom, en: Enumeration, f: int, R: int, eb_x0: str = "centroid", eb_bc: str = "dirichlet",
                   wpow: float = 5.0):
    """Rows A~ (N x M), weights W (N), flux vector F~ (M) and the Phi indices of face f,
    in extended precision (see the module notes).

    Rows follow eq. 'volume moment eq for cp' (volume averages: A_vp = m^p_v(x0)/m^0_v)
    and eq. 'Dir moment eq for cp' (Dirichlet boundary faces: b_p = m^p(x0)/m^0); the
    moments about x0 come from each row's stored moments by the binomial re-centring.
    With eb_bc = "neumann" the EB rows follow eq. 'Neu moment eq for cp' instead
    (b_p = sum_d p_d m^(p-e_d)_d(x0) / m^0, the normal-derivative average; in the scaled
    variables xi = (x - x0)/h this row is h times the physical one).  Box faces are always
    Dirichlet."""
    idx = neighbours(en, f, R)
    x0h = face_centre_h(en, f, eb_x0)
    mom = en.row_mom[idx].astype(LD)            # [N, M]
    delta = en.row_ctr_h[idx].astype(LD) - x0h  # [N, D], (x_i - x0)/h
    A = recentre(mom, delta, en.D, en.Q) / mom[:, :1]
    if eb_bc == "neumann":
        for i, k in enumerate(idx):
            if en.n_vol <= k < en.n_vol + en.n_eb:
                e = int(k - en.n_vol)
                A[i] = eb_normal_flux(geom, en, e, x0h) / LD(geom.eb_mom[e, 0])
    elif eb_bc != "dirichlet":
        raise ValueError(eb_bc)
    W = row_weights(np.sqrt(np.sum(delta * delta, axis=1)), wpow)
    F = flux_vector(geom, en, f, x0h)
    return A, W, F, idx


def face_system(geom, en: Enumeration, f: int, R: int, eb_x0: str = "centroid", eb_bc: str = "dirichlet",
                wpow: float = 5.0):
    """face_system_ld rounded to FP64: rows A~ (N x M), weights W (N), flux vector F~ (M)
    and the Phi indices of face f."""
    A, W, F, idx = face_system_ld(geom, en, f, R, eb_x0, eb_bc, wpow)
    return A.astype(np.float64), W.astype(np.float64), F.astype(np.float64), idx


def householder_qr(B: np.ndarray):
    """Householder QR of B (N x M, N >= M) in the dtype of B, in LAPACK's conventions:
    reflector k is H_k = I - tau_k v_k v_k^T with v_k zero above row k and 1 at row k,
    chosen so that H_k maps the column below the diagonal, x, onto beta_k e_k with
    beta_k = -sign(x_k) ||x|| (tau_k = 0, H_k = I when x has no entries below row k);
    B = H_0 H_1 ... H_{M-1} [R; 0].  Returns (V [N, M], tau [M], R [M, M])."""
    N, M = B.shape
    T = B.dtype.type
    C = B.copy()
    V = np.zeros_like(B)
    tau = np.zeros(M, dtype=B.dtype)
    for k in range(M):
        x = C[k:, k]
        alpha = x[0]
        sigma = np.sqrt(np.sum(x[1:] * x[1:]))
        V[k, k] = 1
        if sigma == 0:
            continue
        beta = -np.copysign(np.sqrt(alpha * alpha + sigma * sigma), alpha)
        tau[k] = (beta - alpha) / beta
        V[k + 1:, k] = x[1:] / (alpha - beta)
        v = V[k:, k]
        C[k:, k + 1:] -= tau[k] * np.outer(v, v @ C[k:, k + 1:])
        C[k, k] = beta
        C[k + 1:, k] = T(0)
    return V, tau, np.triu(C[:M])


def min_norm_solve(V: np.ndarray, tau: np.ndarray, R: np.ndarray, F: np.ndarray) -> np.ndarray:
    """The z of least 2-norm with B^T z = F, from the Householder QR of B: with
    B = Q1 R, B^T z = R^T (Q1^T z), so z = Q1 u with R^T u = F (forward substitution),
    and Q1 u = H_0 ... H_{M-1} [u; 0] (the reflectors applied last to first)."""
    N, M = V.shape
    u = np.zeros(M, dtype=V.dtype)
    for k in range(M):
        u[k] = (F[k] - R[:k, k] @ u[:k]) / R[k, k]
    z = np.zeros(N, dtype=V.dtype)
    z[:M] = u
    for k in range(M - 1, -1, -1):
        v = V[k:, k]
        z[k:] -= tau[k] * v * (v @ z[k:])
    return z


def face_stencil(geom, en: Enumeration, f: int, R: int, eb_x0: str = "centroid", eb_bc: str = "dirichlet",
                 wpow: float = 5.0):
    """Stencil of face f: s = h^(D-2) W (A~^T W)^+ F~ (eq. 'stencil equation solution'),
    the solution of A~^T s~ = F~ of least ||W^-1 s~|| (Sec. 2.2.1): with B = W A~ and
    z = W^-1 s~, z is the minimum-norm solution of B^T z = F~, computed from a Householder
    QR of B with its columns scaled to unit 2-norm (the scaling E changes B^T z = F~ into
    (B E)^T z = E F~, the same z), in extended precision.  Under Neumann EB conditions
    the values of the EB (normal-derivative) rows carry h^(D-1) instead of h^(D-2), and an
    EB face's own flux is its prescribed data: the single entry |A_f| on its Phi entry
    (reading: the paper does not say how the flux of a Neumann face is formed).
    Returns (Phi indices, values, status)."""
    if eb_bc == "neumann" and en.face_kind[f] == KIND_EB:
        e = int(en.face_lin[f])
        return (np.array([en.n_vol + e], np.int64), np.array([geom.eb_mom[e, 0] * en.h ** (en.D - 1)]),
                STATUS_OK)
    A, W, F, idx = face_system_ld(geom, en, f, R, eb_x0, eb_bc, wpow)
    N, M = A.shape
    if not (np.all(np.isfinite(A)) and np.all(np.isfinite(F)) and np.all(np.isfinite(W))):
        return idx, np.zeros(N), STATUS_NONFINITE
    if N < M:
        return idx, np.zeros(N), STATUS_INSUFFICIENT_ROWS
    B = W[:, None] * A
    cn = np.sqrt(np.sum(B * B, axis=0))
    if np.any(cn == 0):
        return idx, np.zeros(N), STATUS_RANK_DEFICIENT
    V, tau, Rm = householder_qr(B / cn)
    r = np.abs(np.diag(Rm))
    if r.min() <= RANK_TOL * r.max():
        return idx, np.zeros(N), STATUS_RANK_DEFICIENT
    z = min_norm_solve(V, tau, Rm, F / cn)
    hs = np.full(N, LD(en.h) ** (en.D - 2), dtype=LD)
    if eb_bc == "neumann":
        hs[(idx >= en.n_vol) & (idx < en.n_vol + en.n_eb)] *= LD(en.h)
    return idx, (hs * W * z).astype(np.float64), STATUS_OK


def face_condition(geom, en: Enumeration, f: int, R: int, eb_bc: str = "dirichlet", wpow: float = 5.0) -> float:
    """2-norm condition number of the column-equilibrated weighted matrix W A~."""
    if eb_bc == "neumann" and en.face_kind[f] == KIND_EB:
        return 1.0
    A, W, F, idx = face_system(geom, en, f, R, eb_bc=eb_bc, wpow=wpow)
    B = W[:, None] * A
    return float(np.linalg.cond(B / np.sqrt(np.sum(B * B, axis=0))))


def build(geom, R: int, faces=None, en: Enumeration | None = None, eb_x0: str = "centroid",
          eb_bc: str = "dirichlet", wpow: float = 5.0):
    """Stencils of all flux faces (or of the listed ones) as CSR arrays
    (row_ptr int64, col int64, val float64, status int8); eb_bc selects Dirichlet or
    Neumann conditions on the embedded boundary (Sec. 2.2.1; box faces stay Dirichlet)."""
    if en is None:
        en = enumerate_geometry(geom)
    fl = range(en.n_face) if faces is None else faces
    rp = [0]
    cols, vals, st = [], [], []
    for f in fl:
        idx, s, status = face_stencil(geom, en, int(f), R, eb_x0, eb_bc, wpow)
        cols.append(idx)
        vals.append(s)
        st.append(status)
        rp.append(rp[-1] + len(idx))
    col = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    val = np.concatenate(vals) if vals else np.zeros(0)
    return en, np.asarray(rp, np.int64), col, val, np.asarray(st, np.int8)


# ---------------------------------------------------------------------------------
# Sec. 2.2 / Sec. 3.3: the operator


def apply(geom, en: Enumeration, row_ptr, col, val, phi):
    """Face fluxes flux_f = s_f^T Phi and the flux divergence
    L_v = (1/|V_v|) sum_{f(v)} sigma_vf flux_f  (Sec. 2.2, eq. 'laplacian over V'),
    with sigma = +1 when the face's reference normal (+e_d for grid faces, out of the
    fluid for EB faces) points out of v (reading R5)."""
    nf = en.n_face
    flux = np.zeros(nf)
    for f in range(nf):
        a, b = row_ptr[f], row_ptr[f + 1]
        flux[f] = np.dot(val[a:b], phi[col[a:b]])
    L = np.zeros(en.n_vol)
    for f in range(nf):
        if en.face_lo[f] >= 0:
            L[en.face_lo[f]] += flux[f]
        if en.face_hi[f] >= 0:
            L[en.face_hi[f]] -= flux[f]
    kappa = geom.vol_mom[en.vol_cell, 0]
    L /= kappa * en.h ** en.D
    return flux, L
