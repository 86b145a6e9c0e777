"""Pins for oracle.rsvd: the SVD of R (Sec. 3.1, R-SVD) and the rank sweep of
residuals in the reduced space (Sec. 2.2, Sec. 2.4)."""

import numpy as np
import pytest

from oracle import nnls, residual, rsvd, select, tsqr


def _rng(*tag):
    return np.random.default_rng([61, *tag])


def test_singular_values_of_r_are_those_of_x():
    """X = QR with Q orthonormal: the singular values of R are those of X, and
    the right singular vectors agree up to sign."""
    X = _rng(1).uniform(size=(3000, 9)) + 0.1
    R = tsqr.tsqr_r_final(X, leaf_rows=512)
    s, U, V = rsvd.rsvd(R)
    sx = np.linalg.svd(X, compute_uv=False)
    assert np.allclose(s, sx, rtol=1e-12)
    _, _, Vx = np.linalg.svd(X, full_matrices=False)
    _, Vx = rsvd.sign_fix(np.zeros((9, 9)), Vx.T)
    assert np.abs(V - Vx).max() <= 1e-9


def test_kronecker_closed_form():
    """sigma(A (x) A) = sigma(A) (x) sigma(A), sorted descending."""
    A = _rng(2).lognormal(size=(40, 4))
    R = tsqr.tsqr_r_final(np.kron(A, A), leaf_rows=200)
    s, _, _ = rsvd.rsvd(R)
    sa = np.linalg.svd(A, compute_uv=False)
    assert np.allclose(s, np.sort(np.kron(sa, sa))[::-1], rtol=1e-11)


def test_reconstruction_orthogonality_and_sign_convention():
    R = np.triu(_rng(3).standard_normal((12, 12)))
    s, U, V = rsvd.rsvd(R)
    assert np.all(np.diff(s) <= 0) and np.all(s >= 0)
    assert np.abs(U @ np.diag(s) @ V.T - R).max() <= 1e-13 * np.abs(R).max()
    assert np.abs(V.T @ V - np.eye(12)).max() <= 1e-13 and np.abs(U.T @ U - np.eye(12)).max() <= 1e-13
    big = np.argmax(np.abs(V), axis=0)
    assert np.all(V[big, np.arange(12)] > 0)


def _separable(m, n, r, seed, noise=0.0):
    rng = _rng(10, seed)
    K = sorted(rng.choice(n, size=r, replace=False).tolist())
    H = rng.dirichlet(np.ones(r), size=n).T
    H[:, K] = np.eye(r)
    X = rng.uniform(size=(m, r)) @ H + noise * rng.uniform(size=(m, n))
    return X, K


@pytest.mark.parametrize("noise", [0.0, 1e-3])
def test_rank_sweep_curve(noise):
    """The residual curve over r = 1..rmax: non-increasing (the picks are
    nested, so each fit has more columns), zero at the planted rank on exactly
    separable data (P8), and equal to the curve computed on X itself (P10)."""
    X, K = _separable(800, 14, 5, 1, noise)
    R = tsqr.tsqr_r_final(X, leaf_rows=256)
    d = np.abs(X).sum(0)
    Ks, res = rsvd.rank_sweep(R, 8, colscale=d)
    assert len(res) == 8
    assert np.all(np.diff(res) <= 1e-15)
    if noise == 0.0:
        assert sorted(Ks[:5]) == K and res[4] <= 1e-24
    else:
        assert res[4] < 1e-5 * res[0]
    for r in (1, 3, 5, 8):
        Hx, _, _ = nnls.nnls_matrix(X, Ks[:r])
        assert abs(residual.relative_residual(X, Ks[:r], Hx) - res[r - 1]) <= 1e-10 * max(res[0], 1e-30)


def test_rank_sweep_matches_spa_prefixes():
    """K of the sweep is SPA's: the picks for rmax start with those for any
    smaller r (SPA is greedy)."""
    X, _ = _separable(500, 12, 4, 2, 1e-3)
    R = tsqr.tsqr_r_final(X, leaf_rows=128)
    d = np.abs(X).sum(0)
    K8, _ = rsvd.rank_sweep(R, 8, colscale=d)
    K3, _, _ = select.spa(R, 3, colscale=d)
    assert K8[:3] == K3
