"""Oracle adjoints: derivatives of the stencils and of the operator apply.

Test infrastructure only (see the package docstring).

The paper defines the forward map only; its derivatives are computed here by
differentiating that definition, step for step:

* ``apply_adjoint``: the transpose of the linear map Phi -> L(Phi) and the derivatives of
  L with respect to the stencil values and the volume fractions (Sec. 2.2,
  eq. 'laplacian over V'), written out directly.
* ``stencils_backward``: the gradient of sum_f sum_j val_bar[j] s_f[j] with respect to
  every input moment (volume, grid-face, EB and EB-normal moments) and to the weights,
  by reverse-mode automatic differentiation (PyTorch on the CPU, FP64) of the same
  steps as ``oracle.stencils``: binomial re-centring of each row's moments to x0
  (Sec. 2.2.1), division by the zeroth moment, the weights of Sec. 2.4 (with x0 of an EB
  face at the centroid of the cut volume, reading R3), the flux vector, and the
  minimum-norm solution of A~^T W y = F~ computed through Householder QR of W A~
  (y = Q R^-T F~).  Integer work (neighbours, enumeration) is taken from the numpy oracle.
"""

from __future__ import annotations

import numpy as np
import torch

from . import stencils as S


def apply_adjoint(geom, en, row_ptr, col, val, phi, lbar):
    """For L(Phi) = D(kappa) (sum over faces of sigma * flux), flux_f = s_f^T Phi:
    returns (phi_bar, val_bar, kappa_bar) = (dl/dPhi, dl/dval, dl/dkappa) for the scalar
    l with dl/dL = lbar."""
    nf = en.n_face
    kappa = geom.vol_mom[en.vol_cell, 0]
    scale = 1.0 / (kappa * en.h**en.D)
    flux, L = S.apply(geom, en, row_ptr, col, val, phi)
    # dl/dflux_f = sum_v sigma_vf lbar_v scale_v
    c = np.zeros(nf)
    for f in range(nf):
        if en.face_lo[f] >= 0:
            c[f] += lbar[en.face_lo[f]] * scale[en.face_lo[f]]
        if en.face_hi[f] >= 0:
            c[f] -= lbar[en.face_hi[f]] * scale[en.face_hi[f]]
    phi_bar = np.zeros(en.n_phi)
    val_bar = np.zeros(len(val))
    for f in range(nf):
        a, b = row_ptr[f], row_ptr[f + 1]
        np.add.at(phi_bar, col[a:b], val[a:b] * c[f])
        val_bar[a:b] = c[f] * phi[col[a:b]]
    kappa_bar = -lbar * L / kappa          # L_v is proportional to 1/kappa_v
    return phi_bar, val_bar, kappa_bar


# ---------------------------------------------------------------------------------
# stencil gradients by automatic differentiation of the definition


def _recentre_t(mom, delta, D, Q):
    coef, ex, qi, P = S._shift_terms(D, Q)
    coef = torch.as_tensor(coef)
    ex = torch.as_tensor(ex, dtype=torch.float64)
    Pm = torch.as_tensor(P)
    powers = torch.prod(delta.unsqueeze(-2) ** ex, dim=-1)          # [..., T]
    return (coef * powers * mom[..., qi]) @ Pm


class _Rows:
    """Leaf tensors for the rows of one input array that one face reads, made on first use
    (the gradient of a face touches only those rows, so it is formed on them and added into
    the full-size gradient afterwards)."""

    def __init__(self, arr, grad=True):
        self.arr = arr
        self.grad = grad
        self.leaves = {}

    def __getitem__(self, key):
        i, rest = (int(key[0]), key[1:]) if isinstance(key, tuple) else (int(key), ())
        t = self.leaves.get(i)
        if t is None:
            t = torch.tensor(np.asarray(self.arr[i]), dtype=torch.float64, requires_grad=self.grad)
            self.leaves[i] = t
        return t[rest] if rest else t

    def add_grad_to(self, out):
        for i, t in self.leaves.items():
            if t.grad is not None:
                out[i] += t.grad.numpy()


class _Inputs:
    """The inputs the stencils read: volume, grid-face, EB and EB-normal moments, as leaf
    rows (grad=True) or constant rows."""

    def __init__(self, geom, grad=True):
        self.vol = _Rows(geom.vol_mom, grad)
        self.face = [_Rows(fm, grad) for fm in geom.face_mom]
        self.eb = _Rows(geom.eb_mom, grad)
        self.ebn = _Rows(geom.eb_nmom, grad)


def _row_moments(inp, en, idx):
    """Each row's moments about its own centre (as in oracle.stencils) from the leaves."""
    D, Q = en.D, en.Q
    mono = S._mono(D, Q)
    rows = []
    for k in idx:
        k = int(k)
        if k < en.n_vol:
            rows.append(inp.vol[int(en.vol_cell[k])])
        elif k < en.n_vol + en.n_eb:
            rows.append(inp.eb[k - en.n_vol])
        else:
            b = k - en.n_vol - en.n_eb
            d, flin = int(en.box_dir[b]), int(en.box_face[b])
            monof = {q: i for i, q in enumerate(S._mono(D - 1, Q))}
            parts = []
            for p in mono:
                if p[d] == 0:
                    parts.append(inp.face[d][flin, monof[tuple(p[e] for e in range(D) if e != d)]])
                else:
                    parts.append(torch.zeros((), dtype=torch.float64))
            rows.append(torch.stack(parts))
    return torch.stack(rows)


def _face_stencil_t(inp, en, f, R, wleaf=None, wpow=5.0):
    """Torch version of oracle.stencils.face_stencil (scaled s~, before h^(D-2))."""
    D, Q, h = en.D, en.Q, en.h
    idx = S.neighbours(en, f, R)
    mono = S._mono(D, Q)
    if en.face_kind[f] == S.KIND_EB:
        v = int(en.face_lo[f])
        cv = torch.as_tensor(en.row_ctr[v])
        mv = inp.vol[int(en.vol_cell[v])]
        x0 = cv + h * mv[1: D + 1] / mv[0]
    else:
        x0 = torch.as_tensor(S.face_centre(en, f))
    ctr = torch.as_tensor(en.row_ctr[idx])
    delta = (ctr - x0) / h
    mom = _row_moments(inp, en, idx)
    A = _recentre_t(mom, delta, D, Q) / mom[:, :1]
    dist = torch.sqrt(torch.sum(delta * delta, dim=1))
    W = torch.where(dist < 0.5, torch.ones_like(dist), (2.0 * torch.clamp(dist, min=0.5)) ** -float(wpow))
    if wleaf is not None:
        W = wleaf
    # flux vector about x0
    if en.face_kind[f] == S.KIND_EB:
        e = int(en.face_lin[f])
        c = torch.as_tensor(en.row_ctr[en.n_vol + e])
        nu = _recentre_t(inp.ebn[e], ((c - x0) / h).expand(D, D), D, Q - 1)
        mono1 = {q: i for i, q in enumerate(S._mono(D, Q - 1))}
        F = []
        for p in mono:
            acc = torch.zeros((), dtype=torch.float64)
            for d in range(D):
                if p[d] > 0:
                    q = list(p)
                    q[d] -= 1
                    acc = acc + p[d] * nu[d, mono1[tuple(q)]]
            F.append(acc)
        F = torch.stack(F)
    else:
        d = int(en.face_dir[f])
        monof = {q: i for i, q in enumerate(S._mono(D - 1, Q))}
        F = torch.stack([inp.face[d][int(en.face_lin[f]), monof[tuple(p[k] for k in range(D) if k != d)]]
                         if p[d] == 1 else torch.zeros((), dtype=torch.float64) for p in mono])
    B = W[:, None] * A
    Qf, Rf = torch.linalg.qr(B)
    y = Qf @ torch.linalg.solve_triangular(Rf.T, F[:, None], upper=False)[:, 0]
    return W * y, W, idx


def stencils_backward(geom, en, R, row_ptr, val_bar, faces=None, weights=True, wpow=5.0):
    """Gradient of sum_j val_bar[j] val[j] (val = h^(D-2) s~, the physical stencils) with
    respect to vol_mom, face_mom[d], eb_mom, eb_nmom, and (if `weights`) the weights (per
    nnz, holding the other inputs fixed).  Faces whose status is not OK contribute nothing."""
    fl = range(en.n_face) if faces is None else faces
    hs = en.h ** (en.D - 2)
    w_bar = np.zeros(len(val_bar))
    out = dict(vol_mom=np.zeros(geom.vol_mom.shape), face_mom=[np.zeros(fm.shape) for fm in geom.face_mom],
               eb_mom=np.zeros(np.shape(geom.eb_mom)), eb_nmom=np.zeros(np.shape(geom.eb_nmom)))
    for f in fl:
        f = int(f)
        a, b = int(row_ptr[f]), int(row_ptr[f + 1])
        vb = torch.as_tensor(val_bar[a:b])
        if not np.any(val_bar[a:b]):
            continue
        idx0, s0, status = S.face_stencil(geom, en, f, R, wpow=wpow)
        if status != S.STATUS_OK:
            continue
        inp = _Inputs(geom)
        s, W, idx = _face_stencil_t(inp, en, f, R, wpow=wpow)
        obj = hs * torch.sum(vb * s)
        if obj.requires_grad:
            obj.backward()
        inp.vol.add_grad_to(out["vol_mom"])
        for d in range(len(inp.face)):
            inp.face[d].add_grad_to(out["face_mom"][d])
        inp.eb.add_grad_to(out["eb_mom"])
        inp.ebn.add_grad_to(out["eb_nmom"])
        if not weights:
            continue
        # weights as free leaves: d/dW of the same objective
        wl = W.detach().clone().requires_grad_(True)
        s_w, _, _ = _face_stencil_t(_Inputs(geom, grad=False), en, f, R, wleaf=wl, wpow=wpow)
        gw, = torch.autograd.grad(hs * torch.sum(vb * s_w), wl)
        w_bar[a:b] = gw.numpy()
    out["weight"] = w_bar
    return out
