"""Oracle: R factor of the thin QR of a tall-and-skinny X (test infrastructure).

Sec. 3.1 defines the thin QR X = QR (Q m x n with orthonormal columns, R n x n
upper triangular) and notes that only R is needed, Q^T being applied
implicitly; TSQR computes it from QR factorisations of row blocks whose R
factors are stacked and factored again (the map and reduce stages of Sec. 3.5).
Sec. 3.3 adds the column norms, accumulated in the same pass.

This module restates those steps plainly in FP64:
  householder_r   one Householder QR (LAPACK dgeqrf convention), R only.
  tsqr_r          leaves of height b, then a binary tree of stacked-R QRs.
  finalize        flip rows so that diag(R) >= 0, zero the strict lower part.
  reference_sums  l1 column sums, squared column 2-norms and X^T X, accumulated
                  by row chunks with a long-double running sum.
"""

import numpy as np


def householder_r(A):
    """R factor (n x n, upper) of one Householder QR of A (b x n), Q discarded.

    Sec. 3.1: thin QR, R only.  The reflector for column j is built the LAPACK
    way: alpha = A[j, j], sigma = ||A[j+1:, j]||_2; if sigma = 0 the reflector is
    the identity (tau = 0, beta = alpha); otherwise
        beta = -sign(alpha) * hypot(alpha, sigma)   (sign(0) = +1),
        tau  = (beta - alpha) / beta,
        v    = [1; A[j+1:, j] / (alpha - beta)],
    and the trailing columns are updated as A -= tau * v (v^T A).
    A block with fewer rows than columns is padded with zero rows (zero rows do
    not change R).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    if A.ndim != 2:
        raise ValueError("A must be 2-D")
    b, n = A.shape
    if b < n:
        A = np.vstack([A, np.zeros((n - b, n))])
        b = n
    for j in range(n):
        x = A[j:, j]
        alpha = x[0]
        sigma = np.linalg.norm(x[1:]) if x.shape[0] > 1 else 0.0
        if sigma == 0.0:
            A[j + 1:, j] = 0.0
            continue
        beta = -np.copysign(np.hypot(alpha, sigma), alpha)
        tau = (beta - alpha) / beta
        v = x / (alpha - beta)
        v[0] = 1.0
        if j + 1 < n:
            w = v @ A[j:, j + 1:]
            A[j:, j + 1:] -= tau * np.outer(v, w)
        A[j, j] = beta
        A[j + 1:, j] = 0.0
    return np.triu(A[:n, :])


def tsqr_r(X, leaf_rows=1000):
    """TSQR R factor: Householder QR of each row block, then a binary tree.

    Sec. 3.1 / Sec. 3.5: each leaf (row block of height ``leaf_rows``; the last
    one may be shorter) is factored on its own; the list of n x n factors is
    then reduced pairwise, each pair being replaced by the R of the stacked
    2n x n matrix; an odd last element moves up a level unchanged.  Any tree
    gives the same R up to row signs and rounding, so the shape is a free
    choice of the implementation.
    """
    X = np.asarray(X)
    m, n = X.shape
    if m < 1 or n < 1:
        raise ValueError("empty matrix")
    return reduce_tree(leaf_factors(X, leaf_rows))


def leaf_factors(X, leaf_rows):
    """The leaf step: the R of every row block of height ``leaf_rows``."""
    X = np.asarray(X)
    return [householder_r(np.asarray(X[i:i + leaf_rows], dtype=np.float64))
            for i in range(0, X.shape[0], leaf_rows)]


def reduce_tree(level):
    """The binary tree: pairs (0, 1), (2, 3), ... of a level are replaced by the
    R of their stacked 2n x n matrix; an odd last factor moves up unchanged."""
    level = list(level)
    while len(level) > 1:
        nxt = []
        for t in range(0, len(level) - 1, 2):
            nxt.append(householder_r(np.vstack([level[t], level[t + 1]])))
        if len(level) % 2 == 1:
            nxt.append(level[-1])
        level = nxt
    return level[0]


def finalize(R):
    """Unique representative: rows with R_ii < 0 are negated (R_ii = 0 counts as
    positive), and the strictly lower triangle is exactly zero."""
    R = np.triu(np.array(R, dtype=np.float64, copy=True))
    neg = np.diag(R) < 0
    R[neg, :] = -R[neg, :]
    return R


def tsqr_r_final(X, leaf_rows=1000):
    """tsqr_r followed by finalize: the R the library is asked to return."""
    return finalize(tsqr_r(X, leaf_rows))


def reference_sums(X, chunk=1 << 16):
    """Reference quantities accumulated over row chunks.

    Returns (colsum_l1, colnorm2_sq, gram):
      colsum_l1[j]   = sum_i |X_ij|   (the diagonal of D in Sec. 3.3; l1 because
                       Sec. 2.1 and Sec. 2.3 normalise columns to sum to one),
      colnorm2_sq[j] = sum_i X_ij^2   (preserved by Q^T, Sec. 2.2),
      gram           = X^T X          (equal to R^T R for the thin QR).
    Products of FP32 data are exact in FP64; each chunk is summed in FP64 and
    the chunk results are added in long double.
    """
    X = np.asarray(X)
    m, n = X.shape
    s1 = np.zeros(n, dtype=np.longdouble)
    s2 = np.zeros(n, dtype=np.longdouble)
    g = np.zeros((n, n), dtype=np.longdouble)
    for i in range(0, m, chunk):
        C = np.asarray(X[i:i + chunk], dtype=np.float64)
        s1 += np.abs(C).sum(axis=0).astype(np.longdouble)
        s2 += (C * C).sum(axis=0).astype(np.longdouble)
        g += (C.T @ C).astype(np.longdouble)
    return s1.astype(np.float64), s2.astype(np.float64), g.astype(np.float64)


def reference_sums_exact(X):
    """Long-double accumulation row by row, for small inputs (pins the chunked
    version and serves the FP64-path tolerance checks)."""
    C = np.asarray(X, dtype=np.longdouble)
    s1 = np.abs(C).sum(axis=0)
    s2 = (C * C).sum(axis=0)
    g = C.T @ C
    return s1.astype(np.float64), s2.astype(np.float64), g.astype(np.float64)
