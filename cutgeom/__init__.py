"""Seeded synthetic inputs for the cut-cell flux-stencil library.

This package is the input generator shared by the oracle, the tests and the benchmark.
It holds none of the stencil method's arithmetic: it produces the geometry (volume,
face and embedded-boundary moments from host quadrature of a level set), analytic test
fields and their exact integrals, and the seeded random fields of the workloads.

Conventions (the library header states the same ones):

* Cells are indexed linearly with x fastest: ``c = i0 + n0*(i1 + n1*i2)``.
* Grid faces of direction ``d`` live on a lattice with ``n_d + 1`` points along ``d``;
  face ``j`` lies on the plane ``x_d = j_d h`` between cells ``j - e_d`` and ``j``.
* Monomials are graded (total degree ascending); inside a degree the first exponent
  descends, then the second, ... (the last varies fastest).
* Moments are scaled: coordinates ``(x - c)/h`` about the Cartesian cell (face) centre,
  integrals divided by ``h^D`` (cells) or ``h^(D-1)`` (faces and EB faces).  Hence the
  zeroth cell moment is the volume fraction kappa and the zeroth face moment is the
  area fraction alpha.
* EB normals point out of the fluid.
"""

from __future__ import annotations

import ctypes
import math
import os
import subprocess
from dataclasses import dataclass, field
from math import comb

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cutgeom.cpp")
_LIB = os.path.join(_HERE, "_cutgeom.so")

BALL, HALFSPACE, STAR2, SH3 = range(4)


def build(force: bool = True) -> str:
    """Compile the host quadrature library in place (g++, OpenMP)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + ".tmp"
        subprocess.check_call(
            ["g++", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c++17", "-o", tmp, _SRC]
        )
        os.replace(tmp, _LIB)
    return _LIB


_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build(force=True)
        lib = ctypes.CDLL(_LIB)
        P = ctypes.c_void_p
        lib.cg_classify.restype = ctypes.c_long
        lib.cg_classify.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, P]
        lib.cg_geometry.restype = ctypes.c_long
        lib.cg_geometry.argtypes = [
            ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int, ctypes.c_int,
            P, P, ctypes.c_long, P, P, P, P, P, P, P,
        ]
        lib.cg_integrate.restype = ctypes.c_long
        lib.cg_integrate.argtypes = [
            ctypes.c_int, ctypes.c_int, P, ctypes.c_int, P, ctypes.c_double, ctypes.c_int,
            P, P, ctypes.c_long, ctypes.c_int, ctypes.c_int, P, P, P, P, P, P, P, P, P, P, P, P, P,
        ]
        lib.cg_psi.restype = ctypes.c_int
        lib.cg_psi.argtypes = [ctypes.c_int, ctypes.c_int, P, ctypes.c_int, ctypes.c_long, P, P]
        _lib = lib
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


# ---------------------------------------------------------------------------------
# monomials


def monomials(D: int, Q: int) -> list[tuple[int, ...]]:
    """Exponents of the monomials of degree <= Q in D variables, in graded order."""
    out = []
    for g in range(Q + 1):
        if D == 1:
            out.append((g,))
        elif D == 2:
            for a in range(g, -1, -1):
                out.append((a, g - a))
        else:
            for a in range(g, -1, -1):
                for b in range(g - a, -1, -1):
                    out.append((a, b, g - a - b))
    return out


def n_monomials(D: int, Q: int) -> int:
    return comb(Q + D, D)


# ---------------------------------------------------------------------------------
# shapes: the fluid is {psi > 0}


@dataclass(frozen=True)
class Shape:
    kind: int
    dim: int
    params: tuple

    def psi(self, x: np.ndarray) -> np.ndarray:
        x = np.ascontiguousarray(np.atleast_2d(x), dtype=np.float64)
        pts = np.zeros((x.shape[0], 3))
        pts[:, : x.shape[1]] = x
        out = np.empty(x.shape[0])
        p = np.asarray(self.params, dtype=np.float64)
        rc = _load().cg_psi(self.kind, self.dim, _ptr(p), len(p), x.shape[0], _ptr(pts), _ptr(out))
        if rc != 0:
            raise ValueError("bad shape")
        return out


def ball_outside(center, r) -> Shape:
    c = list(center) + [0.0] * (3 - len(center))
    return Shape(BALL, len(center), tuple(c) + (float(r), 1.0))


def ball_inside(center, r) -> Shape:
    c = list(center) + [0.0] * (3 - len(center))
    return Shape(BALL, len(center), tuple(c) + (float(r), -1.0))


def halfspace(normal, offset) -> Shape:
    """Fluid is {normal . x > offset}."""
    nvec = list(normal) + [0.0] * (3 - len(normal))
    return Shape(HALFSPACE, len(normal), tuple(nvec) + (float(offset), 1.0))


def star2_outside(center, r0, amp, k) -> Shape:
    """Outside of the star rho < r0 + amp cos(k theta) about ``center`` (2D)."""
    return Shape(STAR2, 2, (center[0], center[1], float(r0), float(amp), float(k), 1.0))


def sh_body_outside(center, r0, coef) -> Shape:
    """Outside of the body rho < r0 + sum_j coef[j] Y_j (real orthonormal spherical
    harmonics, l <= 3, ordered (l, m = -l..l))."""
    coef = np.asarray(coef, dtype=np.float64)
    assert coef.shape == (16,)
    return Shape(SH3, 3, tuple(center) + (float(r0),) + tuple(coef.tolist()) + (1.0,))


def perturbed_spheres(n_geom=64, seed=3) -> list:
    """The batched workload's shapes: unit cubes minus spheres with centres
    0.5 + U(-0.05, 0.05)^3 and radii U(0.25, 0.35), drawn from default_rng(seed), all
    centres first, then all radii."""
    rng = np.random.default_rng(seed)
    centres = 0.5 + rng.uniform(-0.05, 0.05, (n_geom, 3))
    radii = rng.uniform(0.25, 0.35, n_geom)
    return [ball_outside(tuple(float(v) for v in c), float(r)) for c, r in zip(centres, radii)]


# ---------------------------------------------------------------------------------
# geometry


@dataclass
class Geometry:
    """Dense cut-cell geometry on the unit box [0,1]^D with ``n`` cells per side."""

    shape: Shape
    D: int
    n: tuple
    h: float
    Q: int
    state: np.ndarray        # int8 [ncell]: 0 covered, 1 full, 2 cut
    vol_mom: np.ndarray      # [ncell, M]
    face_mom: list           # D arrays [nface_d, Mf]
    eb_cell: np.ndarray      # int32 [n_eb], ascending
    eb_mom: np.ndarray       # [n_eb, M]
    eb_nmom: np.ndarray      # [n_eb, D, M1]
    qorder: int = 10
    cand: np.ndarray = field(default=None, repr=False)     # candidate cells (int64)
    eb_pos: np.ndarray = field(default=None, repr=False)   # candidate slot of each EB face

    @property
    def ncell(self) -> int:
        return int(np.prod(self.n))

    @property
    def M(self) -> int:
        return n_monomials(self.D, self.Q)

    @property
    def Mf(self) -> int:
        return n_monomials(self.D - 1, self.Q)

    @property
    def M1(self) -> int:
        return n_monomials(self.D, self.Q - 1)

    def face_dims(self, d: int) -> tuple:
        m = list(self.n)
        m[d] += 1
        return tuple(m)

    @property
    def kappa(self) -> np.ndarray:
        return self.vol_mom[:, 0]

    def alpha(self, d: int) -> np.ndarray:
        return self.face_mom[d][:, 0]

    # ---- Phi layout convention ------------------------------------------------
    def box_faces(self) -> list:
        """Box faces with alpha > 0 in Phi order: by (d, side, adjacent cell index).
        Returns a list of (d, side, face_linear_index, cell_linear_index)."""
        out = []
        for d in range(self.D):
            m = self.face_dims(d)
            for side in (0, 1):
                # cells adjacent to the side, ascending linear cell index
                cells = np.arange(self.ncell)
                idx = np.unravel_index(cells, self.n, order="F")
                on = idx[d] == (0 if side == 0 else self.n[d] - 1)
                cells = cells[on]
                ii = [a[on] for a in idx]
                jj = list(ii)
                if side == 1:
                    jj[d] = jj[d] + 1
                f = np.ravel_multi_index(tuple(jj), m, order="F")
                keep = self.face_mom[d][f, 0] > 0
                for fi, ci in zip(f[keep], cells[keep]):
                    out.append((d, side, int(fi), int(ci)))
        return out

    def phi_counts(self) -> tuple:
        n_vol = int(np.count_nonzero(self.kappa > 0))
        return n_vol, len(self.eb_cell), len(self.box_faces())

    def layout_phi(self, vol_val: np.ndarray, eb_val: np.ndarray, face_val: list) -> np.ndarray:
        """Arrange dense values into the Phi vector [volumes | EB faces | box faces]."""
        vols = np.nonzero(self.kappa > 0)[0]
        parts = [vol_val[vols], eb_val]
        box = self.box_faces()
        parts.append(np.array([face_val[d][f] for (d, s, f, c) in box], dtype=np.float64))
        return np.concatenate(parts)

    # ---- exact integrals of analytic fields ----------------------------------
    def integrate(self, field) -> dict:
        """Exact (quadrature) integrals of ``field`` over the geometry (physical units)."""
        lib = _load()
        p = np.asarray(self.shape.params, dtype=np.float64)
        nn = np.array(list(self.n) + [1] * (3 - self.D), dtype=np.int32)
        nc = self.ncell
        vol_int = np.zeros(nc)
        vol_lap = np.zeros(nc)
        fi = [np.zeros(int(np.prod(self.face_dims(d)))) for d in range(self.D)]
        ff = [np.zeros(int(np.prod(self.face_dims(d)))) for d in range(self.D)]
        while len(fi) < 3:
            fi.append(None)
            ff.append(None)
        ncand = len(self.cand)
        eb_int = np.zeros(max(ncand, 1))
        eb_flux = np.zeros(max(ncand, 1))
        amp, om, ph = field.packed(self.D)
        state = np.ascontiguousarray(self.state)
        nerr = lib.cg_integrate(
            self.shape.kind, self.D, _ptr(p), len(p), _ptr(nn), self.h, self.qorder,
            _ptr(state), _ptr(self.cand), ncand, field.KIND, len(amp), _ptr(amp), _ptr(om), _ptr(ph),
            _ptr(vol_int), _ptr(vol_lap), _ptr(fi[0]), _ptr(fi[1]), _ptr(fi[2]),
            _ptr(ff[0]), _ptr(ff[1]), _ptr(ff[2]), _ptr(eb_int), _ptr(eb_flux),
        )
        if nerr != 0:
            raise RuntimeError(f"quadrature failures: {nerr}")
        return dict(
            vol_int=vol_int, vol_lap=vol_lap, face_int=fi[: self.D], face_flux=ff[: self.D],
            eb_int=eb_int[self.eb_pos], eb_flux=eb_flux[self.eb_pos],
        )


def make_geometry(shape: Shape, n, Q: int, qorder: int = 10) -> Geometry:
    """Volume, face and EB moments of the fluid {psi > 0} on the unit box with ``n``
    cells per direction (host quadrature of the level set)."""
    lib = _load()
    D = shape.dim
    n = tuple(int(v) for v in (n if np.iterable(n) else [n] * D))
    assert len(n) == D
    h = 1.0 / n[0]
    assert all(abs(1.0 / v - h) < 1e-15 for v in n), "square cells only"
    nn = np.array(list(n) + [1] * (3 - D), dtype=np.int32)
    p = np.asarray(shape.params, dtype=np.float64)
    ncell = int(np.prod(n))
    state = np.empty(ncell, dtype=np.int8)
    ncand = lib.cg_classify(shape.kind, D, _ptr(p), len(p), _ptr(nn), h, _ptr(state))
    if ncand < 0:
        raise ValueError("bad shape parameters")
    cand = np.nonzero(state == 2)[0].astype(np.int64)
    M = n_monomials(D, Q)
    Mf = n_monomials(D - 1, Q)
    M1 = n_monomials(D, Q - 1)
    vol_mom = np.empty((ncell, M))
    fm = []
    for d in range(D):
        m = list(n)
        m[d] += 1
        fm.append(np.empty((int(np.prod(m)), Mf)))
    fptr = [_ptr(a) for a in fm] + [None] * (3 - D)
    nc = max(len(cand), 1)
    eb_mom = np.zeros((nc, M))
    eb_nmom = np.zeros((nc, D, M1))
    eb_area = np.zeros(nc)
    nerr = lib.cg_geometry(
        shape.kind, D, _ptr(p), len(p), _ptr(nn), h, Q, qorder, _ptr(state), _ptr(cand), len(cand),
        _ptr(vol_mom), fptr[0], fptr[1], fptr[2], _ptr(eb_mom), _ptr(eb_nmom), _ptr(eb_area),
    )
    if nerr != 0:
        raise RuntimeError(f"quadrature failures: {nerr}")
    keep = np.nonzero(eb_area[: len(cand)] > 0)[0]
    return Geometry(
        shape=shape, D=D, n=n, h=h, Q=Q, state=state, vol_mom=vol_mom, face_mom=fm,
        eb_cell=cand[keep].astype(np.int32), eb_mom=np.ascontiguousarray(eb_mom[keep]),
        eb_nmom=np.ascontiguousarray(eb_nmom[keep]), qorder=qorder, cand=cand, eb_pos=keep,
    )


# ---------------------------------------------------------------------------------
# analytic fields


@dataclass
class TrigField:
    """phi(x) = sum_t amp[t] * prod_d sin(omega[t, d] x_d + phase[t, d])."""

    amp: np.ndarray
    omega: np.ndarray
    phase: np.ndarray
    KIND = 0

    def packed(self, D):
        amp = np.ascontiguousarray(self.amp, dtype=np.float64)
        om = np.zeros((len(amp), 3))
        ph = np.zeros((len(amp), 3))
        om[:, :D] = self.omega
        ph[:, :D] = self.phase
        return amp, om, ph

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.atleast_2d(x)
        s = np.zeros(x.shape[0])
        for a, w, p in zip(self.amp, self.omega, self.phase):
            s += a * np.prod(np.sin(x * w + p), axis=1)
        return s


def trig_product(omegas, phases, amp=1.0) -> TrigField:
    return TrigField(np.array([amp], float), np.array([omegas], float), np.array([phases], float))


def fourier_field(D: int, kmax: int, rng: np.random.Generator) -> TrigField:
    """phi = sum_{k in [0,kmax]^D} a_k cos(2 pi k.x) + b_k sin(2 pi k.x), a, b ~ N(0,1),
    written as sums of sine products (cos(u+v) = sin(u+pi/2)sin(v+pi/2) - sin(u)sin(v))."""
    assert D == 2
    ab = rng.standard_normal((kmax + 1, kmax + 1, 2))
    amp, om, ph = [], [], []
    tp = 2 * math.pi
    h = math.pi / 2
    for kx in range(kmax + 1):
        for ky in range(kmax + 1):
            a, b = ab[kx, ky]
            w = (tp * kx, tp * ky)
            # a cos(u + v) = a [cos u cos v - sin u sin v]
            amp += [a, -a]
            om += [w, w]
            ph += [(h, h), (0.0, 0.0)]
            # b sin(u + v) = b [sin u cos v + cos u sin v]
            amp += [b, b]
            om += [w, w]
            ph += [(0.0, h), (h, 0.0)]
    return TrigField(np.array(amp), np.array(om), np.array(ph))


@dataclass
class PolyField:
    """phi(x) = sum_t amp[t] * prod_d (x_d - xref_d)^expo[t, d]."""

    amp: np.ndarray
    expo: np.ndarray
    xref: np.ndarray
    KIND = 1

    def packed(self, D):
        amp = np.ascontiguousarray(self.amp, dtype=np.float64)
        om = np.zeros((len(amp), 3))
        ph = np.zeros((len(amp), 3))
        om[:, :D] = self.expo
        ph[0, :D] = self.xref
        return amp, om, ph

    def __call__(self, x: np.ndarray) -> np.ndarray:
        x = np.atleast_2d(x)
        s = np.zeros(x.shape[0])
        for a, e in zip(self.amp, self.expo):
            s += a * np.prod((x - self.xref) ** e, axis=1)
        return s


def random_polynomial(D: int, degree: int, rng: np.random.Generator, xref=None, scale=1.0) -> PolyField:
    """A polynomial of total degree <= ``degree`` with N(0,1) coefficients in the
    variables (x - xref)/scale."""
    mono = monomials(D, degree)
    c = rng.standard_normal(len(mono))
    xref = np.full(D, 0.5) if xref is None else np.asarray(xref, float)
    amp = np.array([ci / scale ** sum(p) for ci, p in zip(c, mono)])
    return PolyField(amp, np.array(mono, dtype=float), xref)
