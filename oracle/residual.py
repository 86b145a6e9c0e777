"""Oracle: relative residual of a separable factorisation (test infrastructure).

Sec. 4 reports ||X - X(:, K) H||_F^2 / ||X||_F^2.  Sec. 2.4 notes that each
column's residual is the same when posed on R, so the ratio can be computed
from the n x n factor alone.
"""

import numpy as np


def relative_residual(M, K, H):
    """||M - M(:, K) H||_F^2 / ||M||_F^2 for any M (X itself or its R)."""
    M = np.asarray(M, dtype=np.float64)
    H = np.asarray(H, dtype=np.float64)
    E = M - M[:, list(K)] @ H
    den = float(np.sum(M * M))
    return float(np.sum(E * E)) / den if den > 0 else 0.0
