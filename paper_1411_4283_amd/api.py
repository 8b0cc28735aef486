"""Python binding of libcutcell (torch tensors for device memory and streams).

Every step of the method runs in the HIP library; this module only allocates the
caller-owned buffers the C ABI asks for and passes pointers.
"""

from __future__ import annotations

import ctypes
from dataclasses import dataclass, field
from math import comb

import torch

from . import _lib
from ._lib import (OK, W_NOT_CONVERGED, Geom, GeomGrad, LaplacianArrays, Opts, PackedArrays, PackedSizes, Sizes,
                   StencilArrays, TransposeArrays, Tuning, check, load)


def _ptr(t: torch.Tensor | None) -> int | None:
    return None if t is None else t.data_ptr()


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


@dataclass
class DeviceGeometry:
    """One geometry's moments on the device, in the layouts of include/cutcell.h."""

    dim: int
    n: tuple
    h: float
    order: int
    vol_mom: torch.Tensor           # [ncell, M] float64
    face_mom: list                  # dim tensors [nface_d, Mf] float64
    eb_cell: torch.Tensor           # [n_eb] int32, ascending
    eb_mom: torch.Tensor            # [n_eb, M] float64
    eb_nmom: torch.Tensor           # [n_eb, dim, M1] float64

    @staticmethod
    def from_host(g, device="cuda") -> "DeviceGeometry":
        """From any object with the host arrays (D, n, h, Q, vol_mom, face_mom, eb_cell,
        eb_mom, eb_nmom), e.g. the input generator's geometry."""

        def t(a, dt):
            return torch.as_tensor(a).to(device=device, dtype=dt).contiguous()

        return DeviceGeometry(
            dim=int(g.D), n=tuple(int(v) for v in g.n), h=float(g.h), order=int(g.Q),
            vol_mom=t(g.vol_mom, torch.float64), face_mom=[t(f, torch.float64) for f in g.face_mom],
            eb_cell=t(g.eb_cell, torch.int32), eb_mom=t(g.eb_mom, torch.float64),
            eb_nmom=t(g.eb_nmom, torch.float64),
        )

    def struct(self) -> Geom:
        s = Geom()
        s.vol_mom = _ptr(self.vol_mom)
        for d in range(3):
            s.face_mom[d] = _ptr(self.face_mom[d]) if d < self.dim else None
        s.n_eb = int(self.eb_cell.numel())
        s.eb_cell = _ptr(self.eb_cell)
        s.eb_mom = _ptr(self.eb_mom)
        s.eb_nmom = _ptr(self.eb_nmom)
        return s


_BC = {"dirichlet": _lib.BC_DIRICHLET, "neumann": _lib.BC_NEUMANN}


_FACTOR = {"auto": _lib.FACTOR_AUTO, "qr": _lib.FACTOR_QR, "gram": _lib.FACTOR_GRAM}


def make_opts(dim: int, n, h: float, order: int, path_radius: int, eb_bc: str = "dirichlet",
              reuse_templates: bool = False, weight_power: float | None = None,
              factorization: str = "auto") -> Opts:
    """cutcell_opts; eb_bc: "dirichlet" or "neumann" on every embedded-boundary face;
    reuse_templates: copy the stencils of faces whose systems are bitwise identical;
    weight_power: the exponent p of W = (2d)^-p (None: the paper's 5);
    factorization: "auto" (Gram path, ill-conditioned faces by Householder QR), "qr"
    (every face by Householder QR) or "gram" (every face on the Gram path)."""
    if eb_bc not in _BC:
        raise ValueError(f"eb_bc must be one of {sorted(_BC)}")
    if factorization not in _FACTOR:
        raise ValueError(f"factorization must be one of {sorted(_FACTOR)}")
    o = Opts()
    o.factorization = _FACTOR[factorization]
    o.eb_bc = _BC[eb_bc]
    o.reuse_templates = 1 if reuse_templates else 0
    o.weight_custom = 0 if weight_power is None else 1
    o.weight_power = 5.0 if weight_power is None else float(weight_power)
    o.dim = dim
    nn = list(n) + [1] * (3 - len(n))
    for d in range(3):
        o.n[d] = int(nn[d])
    o.h = float(h)
    o.order = int(order)
    o.path_radius = int(path_radius)
    return o


@dataclass
class Stencils:
    """Build outputs (device tensors) and their sizes."""

    dim: int
    sizes: Sizes
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    status: torch.Tensor
    vol_face: torch.Tensor
    vol_scale: torch.Tensor
    phi_off: torch.Tensor
    vol_off: torch.Tensor
    face_off: torch.Tensor
    tmpl: "torch.Tensor | None" = None   # [n_face] template of each copied face, else -1
    code: int = 0
    reused: int = 0            # faces whose stencil was copied from a template
    qr_faces: int = 0          # faces the Householder QR path solved
    transpose: "Transpose | None" = None
    _keep: list = field(default_factory=list, repr=False)

    def struct(self, val: torch.Tensor | None = None, vol_scale: torch.Tensor | None = None) -> StencilArrays:
        """The C struct; `val` / `vol_scale` replace the stored arrays when given."""
        s = StencilArrays()
        for name in ("row_ptr", "col", "val", "status", "vol_face", "vol_scale", "phi_off", "vol_off", "face_off",
                     "tmpl"):
            setattr(s, name, _ptr(getattr(self, name)))
        if val is not None:
            _check_f64(val, self.sizes.nnz, "val")
            s.val = _ptr(val)
        if vol_scale is not None:
            _check_f64(vol_scale, self.sizes.n_vol, "vol_scale")
            s.vol_scale = _ptr(vol_scale)
        return s


def _check_f64(t: torch.Tensor, n: int, name: str):
    if t.dtype != torch.float64 or not t.is_contiguous() or t.numel() < n or not t.is_cuda:
        raise ValueError(f"{name} must be a contiguous float64 device tensor with at least {n} entries")


@dataclass
class Transpose:
    """Column structure of the stencils (cutcell_build_transpose)."""

    col_ptr: torch.Tensor
    nz: torch.Tensor
    nz_face: torch.Tensor

    def struct(self) -> TransposeArrays:
        s = TransposeArrays()
        s.col_ptr, s.nz, s.nz_face = _ptr(self.col_ptr), _ptr(self.nz), _ptr(self.nz_face)
        return s


def build_transpose(st: Stencils, stream=None) -> Transpose:
    """Transpose of the stencils, cached on `st`."""
    if st.transpose is not None:
        return st.transpose
    s = st.sizes
    dev = st.row_ptr.device
    lib = load()
    nbytes = lib.cutcell_transpose_workspace_bytes(ctypes.byref(s))
    if nbytes == 0:
        raise ValueError("the transpose needs nnz < 2^31")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=dev)
    tr = Transpose(col_ptr=torch.empty(s.n_phi + 1, dtype=torch.int64, device=dev),
                   nz=torch.empty(max(s.nnz, 1), dtype=torch.int32, device=dev),
                   nz_face=torch.empty(max(s.nnz, 1), dtype=torch.int32, device=dev))
    arr, tarr = st.struct(), tr.struct()
    rc = lib.cutcell_build_transpose(ctypes.byref(s), ctypes.byref(arr), ctypes.byref(tarr), _ptr(ws), ws.numel(),
                                     _stream(stream))
    check(rc, "cutcell_build_transpose", allow_flagged=False)
    st.transpose = tr
    st._keep.append(ws)   # the sort's scratch stays alive until the stream has used it
    return tr


def apply_adjoint(st: Stencils, lphi_bar: torch.Tensor, phi: torch.Tensor | None = None,
                  flux: torch.Tensor | None = None, val: torch.Tensor | None = None,
                  vol_scale: torch.Tensor | None = None, stream=None):
    """Adjoint of apply: returns (phi_bar, val_bar or None, scale_bar or None, flux_bar).
    val_bar needs phi; scale_bar needs the forward's flux."""
    s = st.sizes
    dev = lphi_bar.device
    _check_f64(lphi_bar, s.n_vol, "lphi_bar")
    tr = build_transpose(st, stream)
    f64 = dict(dtype=torch.float64, device=dev)
    phi_bar = torch.empty(max(s.n_phi, 1), **f64)
    flux_bar = torch.empty(max(s.n_face, 1), **f64)
    val_bar = torch.empty(max(s.nnz, 1), **f64) if phi is not None else None
    scale_bar = torch.empty(max(s.n_vol, 1), **f64) if flux is not None else None
    arr, tarr = st.struct(val, vol_scale), tr.struct()
    rc = load().cutcell_apply_adjoint(ctypes.byref(s), st.dim, ctypes.byref(arr), ctypes.byref(tarr), _ptr(phi),
                                      _ptr(flux), _ptr(lphi_bar), _ptr(phi_bar), _ptr(val_bar), _ptr(scale_bar),
                                      _ptr(flux_bar), _stream(stream))
    check(rc, "cutcell_apply_adjoint", allow_flagged=False)
    cut = lambda t, n: None if t is None else t[:n]  # noqa: E731
    return phi_bar[: s.n_phi], cut(val_bar, s.nnz), cut(scale_bar, s.n_vol), flux_bar[: s.n_face]


class Builder:
    """Holds the workspace and the ctypes structs of one batch of geometries sharing a
    grid, order and path radius, so repeated builds allocate nothing new."""

    def __init__(self, geoms, path_radius: int, device="cuda", eb_bc: str = "dirichlet",
                 reuse_templates: bool = False, weight_power: float | None = None, factorization: str = "auto"):
        geoms = list(geoms) if isinstance(geoms, (list, tuple)) else [geoms]
        self.tuned_from_cache = False   # the last autotune took every bin from its cache
        g0 = geoms[0]
        for g in geoms:
            assert (g.dim, g.n, g.h, g.order) == (g0.dim, g0.n, g0.h, g0.order), "a batch shares its grid"
        self.geoms = geoms
        self.dim = g0.dim
        self.opts = make_opts(g0.dim, g0.n, g0.h, g0.order, path_radius, eb_bc, reuse_templates, weight_power,
                              factorization)
        self.eb_bc = eb_bc
        self.garr = (Geom * len(geoms))(*[g.struct() for g in geoms])
        lib = load()
        nbytes = lib.cutcell_workspace_bytes(ctypes.byref(self.opts), len(geoms))
        if nbytes == 0:
            raise ValueError("unsupported options")
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        self.device = device
        self.sizes = None
        self.tuning = None

    def set_tuning(self, tuning: "Tuning | None") -> None:
        """Use a launch schedule (from autotune(), or None for the default)."""
        self.tuning = tuning
        self.opts.tuning = ctypes.pointer(tuning) if tuning is not None else None

    def autotune(self, out: "Stencils | None" = None, reps: int = 2, stream=None, cache: str | None = None):
        """Time the candidate launch schedules and kernel widths of every row-count bin on
        these geometries, keep the fastest (set_tuning) and return (tuning, best ms per bin).
        `out` receives the stencils, as from build().

        With `cache` (a JSON file), each bin's choice is kept under the key (GPU
        architecture, D, Q, path radius, bin): when every bin this workload fills has an
        entry, those are used without timing (best ms then -1, and self.tuned_from_cache is
        True); otherwise every bin is timed and the file gets the new entries."""
        if self.sizes is None:
            self.query(stream)
        out = self.allocate() if out is None else out
        self.tuned_from_cache = False
        if cache is not None:
            t = self._tuning_from_cache(cache, out, stream)
            if t is not None:
                self.tuned_from_cache = True
                self.set_tuning(t)
                self.build(out=out, stream=stream)
                return t, [-1.0] * 8
        t = Tuning()
        best = (ctypes.c_double * 8)()
        arr = out.struct()
        rc = load().cutcell_autotune(self.garr, len(self.geoms), ctypes.byref(self.opts), ctypes.byref(self.sizes),
                                     ctypes.byref(arr), _ptr(self.workspace), self.workspace.numel(), int(reps),
                                     ctypes.byref(t), best, _stream(stream))
        out.code = check(rc, "cutcell_autotune")
        self.set_tuning(t)
        best_ms = [best[i] for i in range(8)]
        if cache is not None:
            _cache_store(cache, self._cache_prefix(), t, best_ms)
        return t, best_ms

    def _cache_prefix(self) -> str:
        arch = torch.cuda.get_device_properties(self.device).gcnArchName.split(":")[0]
        return f"{arch}/D{self.dim}/Q{self.opts.order}/R{self.opts.path_radius}"

    def _tuning_from_cache(self, path: str, out: "Stencils", stream) -> "Tuning | None":
        entries = _cache_load(path)
        if not entries:
            return None
        self.set_tuning(None)
        self.build(out=out, stream=stream)   # which bins this workload fills
        counts = (ctypes.c_int64 * 8)()
        load().cutcell_last_bin_faces(counts, 8)
        t = Tuning()
        prefix = self._cache_prefix()
        for b in range(8):
            e = entries.get(f"{prefix}/bin{b}")
            if counts[b] > 0 and e is None:
                return None
            if e is not None:
                t.xcd_chunks[b], t.blocks_per_xcd[b], t.split[b] = e["xcd_chunks"], e["blocks_per_xcd"], e["split"]
        return t

    def query(self, stream=None) -> Sizes:
        sizes = Sizes()
        rc = load().cutcell_query(self.garr, len(self.geoms), ctypes.byref(self.opts), _ptr(self.workspace),
                                  self.workspace.numel(), ctypes.byref(sizes), _stream(stream))
        check(rc, "cutcell_query")
        self.sizes = sizes
        return sizes

    def allocate(self) -> Stencils:
        s = self.sizes if self.sizes is not None else self.query()
        dev = self.device
        G = len(self.geoms)
        i64 = dict(dtype=torch.int64, device=dev)
        return Stencils(
            dim=self.dim, sizes=s,
            row_ptr=torch.empty(s.n_face + 1, **i64),
            col=torch.empty(max(s.nnz, 1), dtype=torch.int32, device=dev),
            val=torch.empty(max(s.nnz, 1), dtype=torch.float64, device=dev),
            status=torch.empty(max(s.n_face, 1), dtype=torch.int8, device=dev),
            vol_face=torch.empty(max(s.n_vol, 1) * (2 * self.dim + 1), dtype=torch.int32, device=dev),
            vol_scale=torch.empty(max(s.n_vol, 1), dtype=torch.float64, device=dev),
            phi_off=torch.empty(G + 1, **i64), vol_off=torch.empty(G + 1, **i64), face_off=torch.empty(G + 1, **i64),
            tmpl=torch.empty(max(s.n_face, 1), dtype=torch.int32, device=dev),
        )

    def build(self, out: Stencils | None = None, stream=None) -> Stencils:
        if self.sizes is None:
            self.query(stream)
        out = self.allocate() if out is None else out
        arr = out.struct()
        rc = load().cutcell_build_stencils(self.garr, len(self.geoms), ctypes.byref(self.opts),
                                           ctypes.byref(self.sizes), ctypes.byref(arr), _ptr(self.workspace),
                                           self.workspace.numel(), _stream(stream))
        out.code = check(rc, "cutcell_build_stencils")
        out.reused = int(load().cutcell_last_reused_faces())
        out.qr_faces = int(load().cutcell_last_qr_faces())
        return out


    def backward(self, st: Stencils, val_bar: torch.Tensor, scale_bar: torch.Tensor | None = None,
                 weight_bar: bool = False, stream=None):
        """Gradients of l with dl/dval = val_bar (and dl/dvol_scale = scale_bar) with respect
        to every geometry's moments: a list of dicts (vol_mom, face_mom, eb_mom, eb_nmom),
        plus weight_bar [nnz] (or None)."""
        s = st.sizes
        _check_f64(val_bar, s.nnz, "val_bar")
        if scale_bar is not None:
            _check_f64(scale_bar, s.n_vol, "scale_bar")
        tr = build_transpose(st, stream)
        lib = load()
        nbytes = lib.cutcell_backward_workspace_bytes(ctypes.byref(self.opts), ctypes.byref(s))
        if nbytes == 0:
            raise ValueError("unsupported options")
        ws = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
        out = []
        garr = (GeomGrad * len(self.geoms))()
        for i, g in enumerate(self.geoms):
            d = dict(vol_mom=torch.empty_like(g.vol_mom), face_mom=[torch.empty_like(f) for f in g.face_mom],
                     eb_mom=torch.empty_like(g.eb_mom), eb_nmom=torch.empty_like(g.eb_nmom))
            out.append(d)
            garr[i].vol_mom = _ptr(d["vol_mom"])
            for k in range(3):
                garr[i].face_mom[k] = _ptr(d["face_mom"][k]) if k < self.dim else None
            garr[i].eb_mom = _ptr(d["eb_mom"]) if d["eb_mom"].numel() else None
            garr[i].eb_nmom = _ptr(d["eb_nmom"]) if d["eb_nmom"].numel() else None
        wb = torch.empty(max(s.nnz, 1), dtype=torch.float64, device=self.device) if weight_bar else None
        arr, tarr = st.struct(), tr.struct()
        rc = lib.cutcell_stencils_backward(self.garr, len(self.geoms), ctypes.byref(self.opts), ctypes.byref(s),
                                           ctypes.byref(arr), ctypes.byref(tarr), _ptr(val_bar), _ptr(scale_bar),
                                           garr, _ptr(wb), _ptr(ws), ws.numel(), _stream(stream))
        check(rc, "cutcell_stencils_backward", allow_flagged=False)
        return out, (None if wb is None else wb[: s.nnz])


def _cache_load(path: str) -> dict:
    import json
    import os

    if not os.path.exists(path):
        return {}
    with open(path) as fh:
        return json.load(fh)


def _cache_store(path: str, prefix: str, t: Tuning, best_ms: list) -> None:
    """Merge the tuned bins (those with a time) into the JSON cache, written atomically."""
    import json
    import os

    entries = _cache_load(path)
    for b in range(8):
        if best_ms[b] >= 0:
            entries[f"{prefix}/bin{b}"] = {"xcd_chunks": int(t.xcd_chunks[b]),
                                           "blocks_per_xcd": int(t.blocks_per_xcd[b]), "split": int(t.split[b]),
                                           "best_ms": float(best_ms[b])}
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as fh:
        json.dump(entries, fh, indent=1, sort_keys=True)
    os.replace(tmp, path)


def build_stencils(geoms, path_radius: int, stream=None, eb_bc: str = "dirichlet") -> Stencils:
    """Flux stencils of every face of one geometry (or a batch sharing a grid)."""
    return Builder(geoms, path_radius, eb_bc=eb_bc).build(stream=stream)


def apply(st: Stencils, phi: torch.Tensor, lphi: torch.Tensor | None = None, flux: torch.Tensor | None = None,
          stream=None, val: torch.Tensor | None = None, vol_scale: torch.Tensor | None = None):
    """L(Phi) = divergence of the face fluxes s_f^T Phi; returns (lphi, flux).  `val` and
    `vol_scale` replace the stencil values and volume scales of `st` when given."""
    s = st.sizes
    assert phi.dtype == torch.float64 and phi.is_contiguous() and phi.numel() == s.n_phi
    if lphi is None:
        lphi = torch.empty(max(s.n_vol, 1), dtype=torch.float64, device=phi.device)
    if flux is None:
        flux = torch.empty(max(s.n_face, 1), dtype=torch.float64, device=phi.device)
    arr = st.struct(val, vol_scale)
    rc = load().cutcell_apply(ctypes.byref(s), st.dim, ctypes.byref(arr), _ptr(phi), _ptr(lphi), _ptr(flux),
                              _stream(stream))
    check(rc, "cutcell_apply", allow_flagged=False)
    return lphi[: s.n_vol], flux[: s.n_face]


@dataclass
class Packed:
    """Compressed stencils (cutcell_pack_*): template-copied faces as a slot plus run bases."""

    sizes: PackedSizes
    flag: torch.Tensor
    phase: torch.Tensor
    face: torch.Tensor
    slot: torch.Tensor
    base: torch.Tensor
    slot_face: torch.Tensor
    slot_rows: torch.Tensor
    slot_tab: torch.Tensor
    slot_val: torch.Tensor

    def struct(self) -> PackedArrays:
        s = PackedArrays()
        for name in ("flag", "phase", "face", "slot", "base", "slot_face", "slot_rows", "slot_tab", "slot_val"):
            setattr(s, name, _ptr(getattr(self, name)))
        return s

    def bytes_per_apply(self) -> int:
        """Bytes the apply reads besides the CSR rows of the other faces: the flags, the
        packed faces' ids, slots, phases and run bases, and the slot tables."""
        p = self.sizes
        return int(self.flag.numel()) + int(p.n_packed) * (9 + 4 * int(p.max_runs)) \
            + int(p.n_slot) * int(p.max_rows) * 12


def pack(st: Stencils, stream=None) -> Packed:
    """Compress the stencils of a build with template reuse (count, then fill)."""
    if st.tmpl is None:
        raise ValueError("the stencils carry no tmpl array")
    s = st.sizes
    dev = st.val.device
    lib = load()
    nbytes = lib.cutcell_pack_workspace_bytes(ctypes.byref(s))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    ps = PackedSizes()
    arr = st.struct()
    check(lib.cutcell_pack_count(ctypes.byref(s), ctypes.byref(arr), ctypes.byref(ps), _ptr(ws), nbytes,
                                 _stream(stream)), "cutcell_pack_count", allow_flagged=False)
    i32 = dict(dtype=torch.int32, device=dev)
    u8 = dict(dtype=torch.uint8, device=dev)
    n, ns = int(ps.n_packed), int(ps.n_slot)
    pk = Packed(ps, torch.empty(max(s.n_face, 1), **u8), torch.empty(max(s.n_face, 1), **u8),
                torch.empty(max(n, 1), **i32), torch.empty(max(n, 1), **i32),
                torch.empty(max(n * ps.max_runs, 1), **i32), torch.empty(max(ns, 1), **i32),
                torch.empty(max(ns, 1), **i32), torch.empty(max(ns * ps.max_rows, 1), **i32),
                torch.empty(max(ns * ps.max_rows, 1), dtype=torch.float64, device=dev))
    pa = pk.struct()
    check(lib.cutcell_pack_fill(ctypes.byref(s), st.dim, ctypes.byref(arr), ctypes.byref(ps), ctypes.byref(pa),
                                _ptr(ws), nbytes, _stream(stream)), "cutcell_pack_fill", allow_flagged=False)
    return pk


def apply_packed(st: Stencils, pk: Packed, phi: torch.Tensor, lphi: torch.Tensor | None = None,
                 flux: torch.Tensor | None = None, stream=None):
    """apply() on the compressed stencils: the same (lphi, flux), bit for bit."""
    s = st.sizes
    _check_f64(phi, s.n_phi, "phi")
    if lphi is None:
        lphi = torch.empty(max(s.n_vol, 1), dtype=torch.float64, device=phi.device)
    if flux is None:
        flux = torch.empty(max(s.n_face, 1), dtype=torch.float64, device=phi.device)
    arr, pa = st.struct(), pk.struct()
    rc = load().cutcell_apply_packed(ctypes.byref(s), st.dim, ctypes.byref(arr), ctypes.byref(pk.sizes),
                                     ctypes.byref(pa), _ptr(phi), _ptr(lphi), _ptr(flux), _stream(stream))
    check(rc, "cutcell_apply_packed", allow_flagged=False)
    return lphi[: s.n_vol], flux[: s.n_face]


@dataclass
class Laplacian:
    """The operator as one sparse matrix over volumes (cutcell_laplacian_*)."""

    dim: int
    sizes: Sizes
    row_ptr: torch.Tensor
    col: torch.Tensor
    val: torch.Tensor
    nnz: int

    def struct(self) -> LaplacianArrays:
        s = LaplacianArrays()
        s.row_ptr, s.col, s.val = _ptr(self.row_ptr), _ptr(self.col), _ptr(self.val)
        return s


def build_laplacian(st: Stencils, stream=None) -> Laplacian:
    """Merge the stencil rows of every volume's faces into its row of L (count, then fill)."""
    s = st.sizes
    dev = st.val.device
    lib = load()
    nbytes = lib.cutcell_laplacian_workspace_bytes(ctypes.byref(s))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=dev)
    row_ptr = torch.empty(s.n_vol + 1, dtype=torch.int64, device=dev)
    nnz = ctypes.c_int64(0)
    arr = st.struct()
    rc = lib.cutcell_laplacian_count(ctypes.byref(s), st.dim, ctypes.byref(arr), _ptr(row_ptr), ctypes.byref(nnz),
                                     _ptr(ws), nbytes, _stream(stream))
    check(rc, "cutcell_laplacian_count", allow_flagged=False)
    n = int(nnz.value)
    lap = Laplacian(st.dim, s, row_ptr, torch.empty(max(n, 1), dtype=torch.int32, device=dev),
                    torch.empty(max(n, 1), dtype=torch.float64, device=dev), n)
    la = lap.struct()
    rc = lib.cutcell_laplacian_fill(ctypes.byref(s), st.dim, ctypes.byref(arr), ctypes.byref(la), _stream(stream))
    check(rc, "cutcell_laplacian_fill", allow_flagged=False)
    return lap


def apply_laplacian(lap: Laplacian, phi: torch.Tensor, lphi: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """L(Phi) through the volume matrix (one gather per volume)."""
    s = lap.sizes
    _check_f64(phi, s.n_phi, "phi")
    if lphi is None:
        lphi = torch.empty(max(s.n_vol, 1), dtype=torch.float64, device=phi.device)
    la = lap.struct()
    rc = load().cutcell_apply_laplacian(ctypes.byref(s), lap.dim, ctypes.byref(la), _ptr(phi), _ptr(lphi),
                                        _stream(stream))
    check(rc, "cutcell_apply_laplacian", allow_flagged=False)
    return lphi[: s.n_vol]


@dataclass
class SolveResult:
    x: torch.Tensor        # volume values of the solution [n_vol]
    iters: int             # Arnoldi steps taken
    relres: float          # final ||b - A x|| / ||b|| (true residual)
    converged: bool


def solve(st: Stencils, phi_bc: torch.Tensor, rhs: torch.Tensor, x0: torch.Tensor | None = None,
          restart: int = 50, max_iters: int = 5000, rtol: float = 1e-10, stream=None,
          lap: "Laplacian | None" = None) -> SolveResult:
    """Solve L([x | bc]) = rhs for the volume values x (cutcell_solve: restarted GMRES with
    right Jacobi preconditioning on the GPU).  `phi_bc` holds the boundary data in its EB
    and box entries; its volume entries are ignored.  With `lap` (build_laplacian of the
    same stencils) the products use the volume matrix."""
    s = st.sizes
    _check_f64(phi_bc, s.n_phi, "phi_bc")
    _check_f64(rhs, s.n_vol, "rhs")
    x = (torch.zeros(max(s.n_vol, 1), dtype=torch.float64, device=phi_bc.device) if x0 is None
         else x0.detach().clone().contiguous())
    _check_f64(x, s.n_vol, "x0")
    nbytes = load().cutcell_solve_workspace_bytes(ctypes.byref(s), restart)
    if nbytes == 0:
        raise ValueError("restart must be in [1, 1024]")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=phi_bc.device)
    it = ctypes.c_int32(0)
    rr = ctypes.c_double(0.0)
    arr = st.struct()
    la = ctypes.byref(lap.struct()) if lap is not None else None
    rc = load().cutcell_solve(ctypes.byref(s), st.dim, ctypes.byref(arr), la, _ptr(phi_bc), _ptr(rhs), _ptr(x),
                              restart, max_iters, rtol, _ptr(ws), nbytes, ctypes.byref(it), ctypes.byref(rr),
                              _stream(stream))
    if rc not in (OK, W_NOT_CONVERGED):
        check(rc, "cutcell_solve", allow_flagged=False)
    return SolveResult(x[: s.n_vol], int(it.value), float(rr.value), rc == OK)


def hessenberg_eigs(H) -> "np.ndarray":
    """Eigenvalues of a square upper Hessenberg matrix (host, cutcell_hessenberg_eigs)."""
    import numpy as np

    H = np.ascontiguousarray(H, dtype=np.float64)
    n = H.shape[0]
    re = np.zeros(max(n, 1))
    im = np.zeros(max(n, 1))
    rc = load().cutcell_hessenberg_eigs(n, H.ctypes.data, H.shape[1], re.ctypes.data, im.ctypes.data)
    check(rc, "cutcell_hessenberg_eigs", allow_flagged=False)
    return (re + 1j * im)[:n]


def ritz(st: Stencils, mode: int = 0, steps: int = 40, lap: "Laplacian | None" = None, inner_rtol: float = 1e-10,
         inner_restart: int = 100, inner_max_iters: int = 5000, stream=None):
    """Ritz values of the volume operator (cutcell_ritz): mode 0 on A (eigenvalues of
    largest magnitude), mode 1 shift-invert about 0 (those nearest 0).  Returns a complex
    numpy array, their relative residuals (small for converged values) and whether every
    inner solve converged."""
    import numpy as np

    s = st.sizes
    lib = load()
    nbytes = lib.cutcell_ritz_workspace_bytes(ctypes.byref(s), steps, mode, inner_restart)
    if nbytes == 0:
        raise ValueError("bad Ritz parameters")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=st.val.device)
    re = np.zeros(steps)
    im = np.zeros(steps)
    res = np.zeros(steps)
    nr = ctypes.c_int32(0)
    arr = st.struct()
    la = ctypes.byref(lap.struct()) if lap is not None else None
    rc = lib.cutcell_ritz(ctypes.byref(s), st.dim, ctypes.byref(arr), la, mode, steps, inner_rtol, inner_restart,
                          inner_max_iters, re.ctypes.data, im.ctypes.data, res.ctypes.data, ctypes.byref(nr),
                          _ptr(ws), nbytes, _stream(stream))
    if rc != W_NOT_CONVERGED:
        check(rc, "cutcell_ritz", allow_flagged=False)
    k = int(nr.value)
    return (re + 1j * im)[:k], res[:k], rc == OK


def n_monomials(dim: int, order: int) -> int:
    return comb(order + dim, dim)
