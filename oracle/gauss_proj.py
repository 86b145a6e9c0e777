"""Oracle: Gaussian projection Y = G^T X (test infrastructure).

Algorithm 1 (Sec. 3.2): the map step forms the outer product g_i x_i^T for each
data row, a combiner sums the outer products of one map task, and the reduce
step sums the partial rows by key.  Whatever the grouping, the result is
Y = sum_i g_i x_i^T = G^T X (k x n).  Sec. 3.3: the column normalisation can be
applied afterwards, (G^T X) D^{-1} = G^T (X D^{-1}).

The oracle sums row chunks in FP64 and adds the chunk results in long double.
"""

import numpy as np

from .philox import gaussian_matrix, gaussian_block


def gauss_proj(X, k, seed, row0=0, chunk=1 << 14):
    """Y (k x n) = G^T X with G from oracle.philox, rows numbered from row0."""
    X = np.asarray(X)
    m, n = X.shape
    Y = np.zeros((k, n), dtype=np.longdouble)
    for i in range(0, m, chunk):
        C = np.asarray(X[i:i + chunk], dtype=np.float64)
        G = gaussian_matrix(seed, row0 + i, C.shape[0], k)
        Y += (G.T @ C).astype(np.longdouble)
    return Y.astype(np.float64)


def gauss_proj_group(X, q, seed, row0=0, chunk=1 << 18):
    """Rows 4q..4q+3 of Y only (one Philox column group), for sampled checks
    at sizes where the full projection would take too long."""
    X = np.asarray(X)
    m, n = X.shape
    Y = np.zeros((4, n), dtype=np.longdouble)
    for i in range(0, m, chunk):
        C = np.asarray(X[i:i + chunk], dtype=np.float64)
        G = gaussian_block(seed, np.arange(row0 + i, row0 + i + C.shape[0], dtype=np.uint64), q)
        Y += (G.T @ C).astype(np.longdouble)
    return Y.astype(np.float64)
