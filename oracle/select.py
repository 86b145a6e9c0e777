"""Oracle: extreme-column selection on the reduced matrices (test
infrastructure).

Sec. 2.2 shows that Q^T X = [R; 0] has the same extreme columns as X, and that
SPA and XRAY only look at column 2-norms, which Q^T preserves; so both can run
on the n x n factor R.  Sec. 3.3 shows that the l1 normalisation X D^{-1}
needed by the convex-hull methods can be applied afterwards as R D^{-1}, and
likewise (G^T X) D^{-1} for the Gaussian projection.

  spa        Successive Projection Algorithm (Sec. 2.1, convex-hull family),
             on M D^{-1} with D = diag(colscale).
  xray       greedy XRAY (Sec. 2.1, conical-hull family) on M itself.
  gp_select  min/max per row of Y D^{-1} (Sec. 2.3).

Ties are broken toward the smallest column index in every argmax/argmin.
"""

import numpy as np

from .nnls import nnls_matrix


def spa(M, r, colscale=None):
    """SPA: r picks of argmax_j ||Z(:, j)||_2^2 with Z the projected residual.

    Sec. 2.1 states the selection rule argmax ||R(:, j)||_2^2 for a residual R
    "related to X"; the residual used here is the standard one of SPA (Araujo et
    al. 2001, cited there): start from Z = M D^{-1}; after picking j*, project
    every column onto the orthogonal complement of Z(:, j*):
        u = Z(:, j*) / ||Z(:, j*)||_2,   Z <- Z - u (u^T Z).
    Already-selected columns are excluded.  If the best score is exactly 0 the
    selection stops early.  Returns (K, scores, info): K in selection order,
    scores the winning ||Z(:, j*)||^2 values, info = number selected.
    """
    M = np.asarray(M, dtype=np.float64)
    p, n = M.shape
    Z = M / np.asarray(colscale, dtype=np.float64)[None, :] if colscale is not None else M.copy()
    K, scores = [], []
    chosen = np.zeros(n, dtype=bool)
    for _ in range(min(r, n)):
        s = np.sum(Z * Z, axis=0)
        s[chosen] = -np.inf
        j = int(np.argmax(s))
        if not s[j] > 0.0:
            break
        K.append(j)
        scores.append(float(s[j]))
        chosen[j] = True
        u = Z[:, j] / np.sqrt(s[j])
        Z = Z - np.outer(u, u @ Z)
    return K, scores, len(K)


def xray(M, r):
    """Greedy XRAY: r picks of argmax_j ||Res^T M(:, j)||_2 / ||M(:, j)||_2.

    Sec. 2.1: the residual Res is updated after each new extreme column.  The
    reading used here: Res starts as M; after each pick Res = M - M(:, K) H with
    H the NNLS fit of every column on the chosen ones (Sec. 2.4's solve).
    Already-chosen and all-zero columns are skipped.  Returns (K, info).
    """
    M = np.asarray(M, dtype=np.float64)
    p, n = M.shape
    norms = np.sqrt(np.sum(M * M, axis=0))
    Res = M.copy()
    K = []
    for _ in range(min(r, n)):
        score = np.full(n, -np.inf)
        for j in range(n):
            if j in K or not norms[j] > 0.0:
                continue
            score[j] = np.linalg.norm(Res.T @ M[:, j]) / norms[j]
        j = int(np.argmax(score))
        if not np.isfinite(score[j]):
            break
        K.append(j)
        H, _, _ = nnls_matrix(M, K)
        Res = M - M[:, K] @ H
    return K, len(K)


def gp_select(Y, r, colscale=None):
    """Gaussian-projection selection (Sec. 2.3).

    For each row of Y D^{-1} the indices of its minimum and maximum entries are
    added to K.  A row contributes up to two indices, so up to 2k distinct
    columns can appear; to return exactly r of them they are ranked by how many
    rows chose them (descending), then by index.  Returns (K, counts, info) with
    info the number returned (fewer than r when fewer distinct columns exist).
    """
    Y = np.asarray(Y, dtype=np.float64)
    k, n = Y.shape
    Yn = Y / np.asarray(colscale, dtype=np.float64)[None, :] if colscale is not None else Y
    counts = np.zeros(n, dtype=np.int64)
    for l in range(k):
        counts[int(np.argmin(Yn[l]))] += 1
        counts[int(np.argmax(Yn[l]))] += 1
    order = sorted([j for j in range(n) if counts[j] > 0], key=lambda j: (-counts[j], j))
    K = order[:r]
    return K, counts, len(K)
