"""The library's host eigensolver for small upper Hessenberg matrices (used for the Ritz
values of the GPU Arnoldi runs), checked without a GPU: against matrices with a known
spectrum (an orthogonal similarity of a block-diagonal matrix with chosen real and
complex-pair eigenvalues, reduced to Hessenberg form by scipy) and against LAPACK on
random Hessenberg matrices."""

import numpy as np
import pytest
import scipy.linalg as sla

import paper_1411_4283_amd as cc


def _match(a, b):
    """Largest distance between two multisets of complex numbers under greedy matching."""
    b = list(b)
    worst = 0.0
    for x in sorted(a, key=lambda z: -abs(z)):
        i = int(np.argmin([abs(x - y) for y in b]))
        worst = max(worst, abs(x - b[i]))
        b.pop(i)
    return worst


def _known(rng, n_real, n_pairs, scale=1.0):
    blocks, lam = [], []
    for _ in range(n_real):
        v = rng.uniform(-1, 1) * scale
        blocks.append(np.array([[v]]))
        lam.append(v)
    for _ in range(n_pairs):
        a, b = rng.uniform(-1, 1) * scale, rng.uniform(0.1, 1) * scale
        blocks.append(np.array([[a, b], [-b, a]]))
        lam += [a + 1j * b, a - 1j * b]
    T = sla.block_diag(*blocks)
    Q, _ = np.linalg.qr(rng.standard_normal(T.shape))
    H = sla.hessenberg(Q @ T @ Q.T)
    return H, np.array(lam)


@pytest.mark.parametrize("n_real,n_pairs", [(1, 0), (0, 1), (2, 0), (5, 3), (20, 10), (60, 20)])
def test_known_spectra(n_real, n_pairs):
    rng = np.random.default_rng(n_real * 100 + n_pairs)
    H, lam = _known(rng, n_real, n_pairs, scale=3.0)
    ev = cc.hessenberg_eigs(H)
    assert len(ev) == len(lam)
    assert _match(ev, lam) <= 1e-11 * np.abs(lam).max()


def test_against_lapack_random_and_operator_like():
    rng = np.random.default_rng(5)
    for n in (3, 10, 40, 100):
        H = np.triu(rng.standard_normal((n, n)), -1)
        ev = cc.hessenberg_eigs(H)
        ref = np.linalg.eigvals(H)
        # random matrices have eigenvalue condition numbers up to ~1e3 at these sizes
        assert _match(ev, ref) <= 1e-9 * np.abs(ref).max(), n
    # spread over seven orders of magnitude, like a cut-cell operator's
    H, lam = _known(rng, 30, 5)
    D = np.diag(np.logspace(0, 7, H.shape[0]))
    H2 = sla.hessenberg(D @ H @ np.linalg.inv(D))
    assert _match(cc.hessenberg_eigs(H2), np.linalg.eigvals(H2)) <= 1e-8 * np.abs(np.linalg.eigvals(H2)).max()


def test_special_cases():
    assert len(cc.hessenberg_eigs(np.zeros((0, 0)))) == 0
    assert cc.hessenberg_eigs(np.array([[2.5]]))[0] == 2.5
    ev = cc.hessenberg_eigs(np.diag([3.0, -1.0, 7.0]))        # already triangular
    assert _match(ev, [3.0, -1.0, 7.0]) == 0.0
    J = np.array([[2.0, 1.0], [0.0, 2.0]])                    # defective
    assert _match(cc.hessenberg_eigs(J), [2.0, 2.0]) <= 1e-8
    R = np.array([[0.0, -1.0], [1.0, 0.0]])                   # rotation: +-i
    assert _match(cc.hessenberg_eigs(R), [1j, -1j]) <= 1e-14
