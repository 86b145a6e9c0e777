"""Pins for oracle.tsqr: the thin-QR R factor (Sec. 3.1) and the reference sums
(Sec. 3.3), checked against things other than the oracle itself."""

import numpy as np
import pytest

from oracle import tsqr


def _rng(*tag):
    return np.random.default_rng([11, *tag])


def _lapack_r(A):
    R = np.linalg.qr(np.asarray(A, dtype=np.float64), mode="r")
    return tsqr.finalize(R)


@pytest.mark.parametrize("m,n", [(1, 1), (3, 1), (5, 5), (8, 3), (17, 4), (64, 8), (40, 7)])
def test_householder_matches_lapack_tiny(m, n):
    """P4: on tiny inputs the oracle's R equals LAPACK's geqrf R after the
    diag >= 0 normalisation."""
    A = _rng(m, n).standard_normal((m, n))
    R = tsqr.finalize(tsqr.householder_r(A))
    ref = _lapack_r(A)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


def test_householder_matches_exact_cholesky_mpmath():
    """The exact R (to 40 digits) is the transposed Cholesky factor of X^T X
    with positive diagonal; small integer matrices make X^T X exact."""
    mpmath = pytest.importorskip("mpmath")
    mpmath.mp.dps = 40
    A = _rng(1).integers(0, 9, size=(9, 4)).astype(np.float64)
    G = mpmath.matrix(A.T.tolist()) * mpmath.matrix(A.tolist())
    L = mpmath.cholesky(G)
    exact = np.array([[float(L[j, i]) for j in range(4)] for i in range(4)])
    R = tsqr.finalize(tsqr.householder_r(A))
    assert np.abs(R - exact).max() <= 1e-14 * np.abs(exact).max()


def test_gram_identity_and_triangular():
    """P1 + P3: R^T R = X^T X, strictly lower part exactly zero, diag >= 0."""
    X = _rng(2).uniform(size=(3000, 13))
    R = tsqr.tsqr_r_final(X, leaf_rows=250)
    G = X.T @ X
    assert np.linalg.norm(R.T @ R - G) / np.linalg.norm(X) ** 2 <= 1e-14
    assert np.all(np.tril(R, -1) == 0.0)
    assert np.all(np.diag(R) >= 0.0)


def test_column_norms_preserved():
    """P2 (Sec. 2.2): ||R(:, j)||_2 = ||X(:, j)||_2."""
    X = _rng(3).lognormal(size=(2000, 9))
    R = tsqr.tsqr_r_final(X, leaf_rows=100)
    assert np.allclose(np.linalg.norm(R, axis=0), np.linalg.norm(X, axis=0), rtol=1e-14, atol=0)


@pytest.mark.parametrize("leaf", [7, 64, 100, 999, 1000, 2500])
def test_tree_invariance(leaf):
    """P5: any leaf height / tree gives the R of a single QR."""
    X = _rng(4).uniform(size=(2500, 11))
    ref = tsqr.finalize(tsqr.householder_r(X))
    R = tsqr.tsqr_r_final(X, leaf_rows=leaf)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


def test_short_leaf_padding():
    """A last leaf shorter than n (here 3 rows for n = 6) is handled by zero rows."""
    X = _rng(5).uniform(size=(103, 6))
    ref = _lapack_r(X)
    R = tsqr.tsqr_r_final(X, leaf_rows=50)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


def test_single_column_closed_form():
    """P6a: n = 1 gives R = ||x||_2."""
    x = _rng(6).uniform(size=(777, 1))
    R = tsqr.tsqr_r_final(x, leaf_rows=100)
    assert R.shape == (1, 1)
    assert abs(R[0, 0] - np.linalg.norm(x)) <= 1e-14 * np.linalg.norm(x)


def test_orthogonal_columns_closed_form():
    """P6b: mutually orthogonal columns give R = diag(column norms)."""
    m, n = 512, 6
    X = np.zeros((m, n))
    s = np.array([3.0, 0.5, 7.0, 1.25, 2.0, 9.0])
    for j in range(n):                  # disjoint row supports -> orthogonal
        X[j * 80:(j + 1) * 80, j] = s[j] / np.sqrt(80.0)
    R = tsqr.tsqr_r_final(X, leaf_rows=64)
    assert np.abs(R - np.diag(s)).max() <= 1e-14 * s.max()


def test_kronecker_closed_form():
    """P6c (Sec. 5.2 builds X = A (x) A): R(A (x) A) = R(A) (x) R(A), and the
    l1 column sums factor the same way."""
    A = _rng(7).lognormal(size=(60, 4))
    X = np.kron(A, A)
    R = tsqr.tsqr_r_final(X, leaf_rows=500)
    RA = _lapack_r(A)
    ref = np.kron(RA, RA)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()
    d, _, _ = tsqr.reference_sums(X)
    dA = np.abs(A).sum(axis=0)
    assert np.allclose(d, np.kron(dA, dA), rtol=1e-14, atol=0)


def test_tiled_copies_closed_form():
    """P6d: X = [A; A; ...; A] (t copies) gives R = sqrt(t) R(A)."""
    A = _rng(8).uniform(size=(37, 5))
    t = 9
    X = np.vstack([A] * t)
    R = tsqr.tsqr_r_final(X, leaf_rows=40)
    ref = np.sqrt(t) * _lapack_r(A)
    assert np.abs(R - ref).max() <= 1e-13 * np.abs(ref).max()


def test_column_scaling_commutes():
    """P11 (Sec. 3.3): R D^{-1} is the R factor of X D^{-1}."""
    X = _rng(9).lognormal(size=(900, 7))
    d, _, _ = tsqr.reference_sums(X)
    R = tsqr.tsqr_r_final(X, leaf_rows=128)
    Rn = tsqr.tsqr_r_final(X / d, leaf_rows=128)
    assert np.abs(R / d - Rn).max() <= 1e-13 * np.abs(Rn).max()


def test_reference_sums_against_exact():
    """Chunked FP64 + long-double sums agree with a long-double row-by-row sum,
    and the l1 sums take absolute values."""
    X = _rng(10).standard_normal((5000, 5))
    a = tsqr.reference_sums(X, chunk=333)
    b = tsqr.reference_sums_exact(X)
    for u, v in zip(a, b):
        assert np.allclose(u, v, rtol=1e-14, atol=1e-14)
    assert np.allclose(a[0], np.abs(X).sum(axis=0), rtol=1e-12)


def test_rank_deficient_gram_still_matches():
    """Z3: exactly separable data with n > r is rank deficient; R is not unique
    beyond rank r, but R^T R = X^T X still holds."""
    rng = _rng(11)
    W = rng.uniform(size=(800, 3))
    H = rng.uniform(size=(3, 8))
    X = W @ H
    R = tsqr.tsqr_r_final(X, leaf_rows=100)
    assert np.linalg.norm(R.T @ R - X.T @ X) / np.linalg.norm(X) ** 2 <= 1e-14
    assert np.all(np.abs(np.diag(R)[3:]) <= 1e-10 * np.abs(R).max())


def test_zero_matrix_and_zero_column():
    X = np.zeros((50, 4))
    assert np.all(tsqr.tsqr_r_final(X, leaf_rows=10) == 0.0)
    X = _rng(12).uniform(size=(60, 4))
    X[:, 2] = 0.0
    R = tsqr.tsqr_r_final(X, leaf_rows=16)
    assert np.all(R[:, 2] == 0.0) or np.abs(R[:, 2]).max() <= 1e-15
    assert np.linalg.norm(R.T @ R - X.T @ X) / np.linalg.norm(X) ** 2 <= 1e-14


def test_parallel_oracle_is_bit_identical():
    """oracle.parallel runs aligned runs of leaves in worker processes and the
    top of the tree in the parent: the same R as tsqr_r, bit for bit, for
    several run sizes and a ragged last leaf and run."""
    from oracle import parallel
    X = np.random.default_rng(91).uniform(size=(13_457, 7)).astype(np.float32)
    ref = tsqr.tsqr_r(X, leaf_rows=1000)
    pool = parallel.OraclePool(2)
    try:
        pool.load(X)
        for run in (None, 1, 2, 4, 16):
            assert np.array_equal(pool.tsqr_r(1000, run_leaves=run), ref)
    finally:
        pool.close()
