"""Pins for the oracle's own rounding error: on well- and ill-conditioned faces its
stencil agrees with a 50-digit evaluation of the same definition from the same FP64
moments (Sec. 2.2.1, eq. 'stencil equation solution'; rows, centring and weights of
Sec. 2.4), to far better than the 1e-11 at which the HIP library is compared with it.

The 50-digit reference forms every derived quantity -- the centroid x0 of an EB face,
the offsets (x_i - x0)/h, the weights, the re-centred rows and flux vector -- from the
moments in mpmath and solves the normal equations s = W^2 A (A^T W^2 A)^-1 F, a
different algorithm from the oracle's Householder QR."""

import math

import mpmath
import numpy as np
import pytest

import cutgeom as cg
import oracle
from oracle import stencils as S

CIRCLE = cg.ball_outside((0.5, 0.5), 0.25)
SPHERE = cg.ball_outside((0.5, 0.5, 0.5), 0.3)


def _monos(D, Q):
    out = []
    for gdeg in range(Q + 1):
        if D == 2:
            out += [(a, gdeg - a) for a in range(gdeg, -1, -1)]
        else:
            out += [(a, b, gdeg - a - b) for a in range(gdeg, -1, -1) for b in range(gdeg - a, -1, -1)]
    return out


def _shift(mom, delta, D, Q):
    """m^p(x0) = sum_{q <= p} prod_d C(p_d, q_d) delta_d^(p_d - q_d) m^q(c) (binomial
    theorem), in mpmath."""
    mono = _monos(D, Q)
    pos = {p: k for k, p in enumerate(mono)}
    out = []
    for p in mono:
        acc = mpmath.mpf(0)
        for q in mono:
            if all(qq <= pp for pp, qq in zip(p, q)):
                t = mom[pos[q]]
                for d in range(D):
                    t *= math.comb(p[d], q[d]) * delta[d] ** (p[d] - q[d])
                acc += t
        out.append(acc)
    return out


def _mp_stencil(g, en, f, R, wpow=5):
    D, Q = g.D, g.Q
    mpmath.mp.dps = 50
    idx = oracle.neighbours(en, f, R)
    mono = _monos(D, Q)
    half = mpmath.mpf(1) / 2
    # x0 / h
    if en.face_kind[f] == S.KIND_EB:
        v = int(en.face_lo[f])
        m = [mpmath.mpf(float(x)) for x in en.row_mom[v]]
        x0 = [mpmath.mpf(float(en.row_ctr_h[v][d])) + m[1 + d] / m[0] for d in range(D)]
    else:
        d0 = int(en.face_dir[f])
        j = np.unravel_index(int(en.face_lin[f]), g.face_dims(d0), order="F")
        x0 = [mpmath.mpf(int(j[d])) + (0 if d == d0 else half) for d in range(D)]
    rows, w2 = [], []
    for k in idx:
        ctr = [mpmath.mpf(float(c)) for c in en.row_ctr_h[k]]
        delta = [ctr[d] - x0[d] for d in range(D)]
        mom = [mpmath.mpf(float(x)) for x in en.row_mom[k]]
        sh = _shift(mom, delta, D, Q)
        rows.append([x / mom[0] for x in sh])
        dist = mpmath.sqrt(sum(x * x for x in delta))
        w = mpmath.mpf(1) if dist < half else (2 * dist) ** (-mpmath.mpf(wpow))
        w2.append(w * w)
    # flux vector
    F = [mpmath.mpf(0)] * len(mono)
    if en.face_kind[f] == S.KIND_EB:
        e = int(en.face_lin[f])
        c = [mpmath.mpf(float(x)) for x in en.row_ctr_h[en.n_vol + e]]
        dl = [c[d] - x0[d] for d in range(D)]
        mono1 = _monos(D, Q - 1)
        pos1 = {p: k for k, p in enumerate(mono1)}
        nu = [_shift([mpmath.mpf(float(x)) for x in g.eb_nmom[e][d]], dl, D, Q - 1) for d in range(D)]
        for a, p in enumerate(mono):
            for d in range(D):
                if p[d] > 0:
                    q = list(p)
                    q[d] -= 1
                    F[a] += p[d] * nu[d][pos1[tuple(q)]]
    else:
        d0 = int(en.face_dir[f])
        fm = g.face_mom[d0][int(en.face_lin[f])]
        tmono = _monos(D - 1, Q) if D == 3 else [(a,) for a in range(Q + 1)]
        tpos = {p: k for k, p in enumerate(tmono)}
        for a, p in enumerate(mono):
            if p[d0] == 1:
                F[a] = mpmath.mpf(float(fm[tpos[tuple(p[d] for d in range(D) if d != d0)]]))
    A = mpmath.matrix(rows)
    W2 = mpmath.diag(w2)
    y = mpmath.lu_solve(A.T * W2 * A, mpmath.matrix(F))
    s = W2 * A * y
    return idx, np.array([float(x) for x in s]) * g.h ** (D - 2)


def _worst_conditioned(g, en, R, wpow, k):
    conds = np.array([oracle.face_condition(g, en, f, R, wpow=wpow) for f in range(en.n_face)])
    return list(np.argsort(conds)[-k:]), conds


@pytest.mark.parametrize("case", ["circle16_q2", "circle16_q4", "sphere8_q4"])
def test_oracle_matches_50_digit_solve(case):
    shape, n, Q, R = {"circle16_q2": (CIRCLE, 16, 2, 2), "circle16_q4": (CIRCLE, 16, 4, 3),
                      "sphere8_q4": (SPHERE, 8, 4, 3)}[case]
    g = cg.make_geometry(shape, n, Q)
    en = oracle.enumerate_geometry(g)
    eb = list(np.flatnonzero(en.face_kind == S.KIND_EB)[:6])
    rest = list(np.random.default_rng(3).choice(en.n_face, 6, replace=False))
    for f in eb + rest:
        idx, s, st = oracle.face_stencil(g, en, int(f), R)
        idx2, se = _mp_stencil(g, en, int(f), R)
        assert np.array_equal(idx, idx2)
        assert np.abs(s - se).max() <= 1e-14 * np.abs(se).max(), (f, np.abs(s - se).max() / np.abs(se).max())


@pytest.mark.slow
def test_oracle_matches_50_digit_solve_on_ill_conditioned_faces():
    """The three worst-conditioned faces of the 32 x 32 circle at fourth order with the
    steep weight exponent 7.5 (cond ~1e6): the oracle is within 1e-12 of the 50-digit
    stencil, so it can decide a 1e-11 comparison on its own; FP64 LAPACK on the FP64
    system is not (its error there is about cond * eps)."""
    g = cg.make_geometry(CIRCLE, 32, 4)
    en = oracle.enumerate_geometry(g)
    faces, conds = _worst_conditioned(g, en, 3, 7.5, 3)
    assert conds[faces].min() > 1e5
    for f in faces:
        idx, s, st = oracle.face_stencil(g, en, int(f), 3, wpow=7.5)
        assert st == oracle.STATUS_OK
        idx2, se = _mp_stencil(g, en, int(f), 3, wpow=7.5)
        err = np.abs(s - se).max() / np.abs(se).max()
        assert err <= 1e-12, (f, err, conds[f])
