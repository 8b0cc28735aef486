"""torch.autograd.Function wrappers of the stencil build and the operator apply, whose
backward passes call the library's hand-written adjoints (cutcell_stencils_backward and
cutcell_apply_adjoint).  Derivatives flow to every moment tensor of the geometries and to
Phi; nothing here computes anything itself.
"""

from __future__ import annotations

import torch

from .api import Builder, apply, apply_adjoint


def _moment_tensors(builder: Builder):
    out = []
    for g in builder.geoms:
        out += [g.vol_mom, *g.face_mom, g.eb_mom, g.eb_nmom]
    return out


class StencilBuild(torch.autograd.Function):
    """(moments of every geometry) -> (val [nnz], vol_scale [n_vol])."""

    @staticmethod
    def forward(ctx, builder: Builder, *moments):
        expect = _moment_tensors(builder)
        if len(moments) != len(expect) or any(a.data_ptr() != b.data_ptr() for a, b in zip(moments, expect)):
            raise ValueError("pass the builder's own moment tensors (the library reads those)")
        st = builder.build()
        builder.last = st
        ctx.builder, ctx.st = builder, st
        s = st.sizes
        return st.val[: s.nnz], st.vol_scale[: s.n_vol]

    @staticmethod
    def backward(ctx, val_bar, scale_bar):
        b, st = ctx.builder, ctx.st
        s = st.sizes
        if val_bar is None:
            val_bar = torch.zeros(s.nnz, dtype=torch.float64, device=st.val.device)
        grads, _ = b.backward(st, val_bar.contiguous(), None if scale_bar is None else scale_bar.contiguous())
        flat = []
        for g in grads:
            flat += [g["vol_mom"], *g["face_mom"], g["eb_mom"], g["eb_nmom"]]
        return (None, *flat)


class OperatorApply(torch.autograd.Function):
    """(val, vol_scale, Phi) -> L(Phi) with the structure of `st`."""

    @staticmethod
    def forward(ctx, st, val, vol_scale, phi):
        lphi, flux = apply(st, phi.contiguous(), val=val, vol_scale=vol_scale)
        lphi, flux = lphi.clone(), flux.clone()
        ctx.st = st
        ctx.save_for_backward(val, vol_scale, phi, flux)
        return lphi

    @staticmethod
    def backward(ctx, lbar):
        val, vol_scale, phi, flux = ctx.saved_tensors
        need = ctx.needs_input_grad
        phi_bar, val_bar, scale_bar, _ = apply_adjoint(
            ctx.st, lbar.contiguous(), phi=phi if need[1] else None, flux=flux if need[2] else None, val=val,
            vol_scale=vol_scale)
        return None, val_bar, scale_bar, (phi_bar if need[3] else None)


class CutCellOperator:
    """L(Phi) for a batch of geometries that share a grid, differentiable with respect to
    Phi and to every moment tensor (set requires_grad on the DeviceGeometry tensors).
    `options` go to the Builder (eb_bc, weight_power, factorization, ...)."""

    def __init__(self, geoms, path_radius: int, **options):
        self.builder = Builder(geoms, path_radius, **options)

    @property
    def geoms(self):
        return self.builder.geoms

    def stencils(self):
        val, scale = StencilBuild.apply(self.builder, *_moment_tensors(self.builder))
        return self.builder.last, val, scale

    def __call__(self, phi: torch.Tensor) -> torch.Tensor:
        st, val, scale = self.stencils()
        return OperatorApply.apply(st, val, scale, phi)
