"""Oracle: nonnegative least squares for the coefficient matrix H (test
infrastructure).

Sec. 2.4: with the extreme columns K chosen, the Frobenius-norm fit splits into
n independent problems  H(:, i) = argmin_{y >= 0} ||X(:, K) y - X(:, i)||_2^2,
and because Q^T preserves 2-norms the same problems can be posed on the n x n
R factor: argmin_{y >= 0} ||R(:, K) y - R(:, i)||_2^2.  The paper does not name
a solver; this oracle uses the classical Lawson-Hanson active-set method
(Lawson & Hanson, "Solving Least Squares Problems", 1974, ch. 23), whose
unconstrained subproblems are solved with a Householder QR (numpy/LAPACK).
When R(:, K) has full column rank the minimiser is unique, so any correct
solver must agree with this one.
"""

import numpy as np


def _ls(A, b):
    """Least-squares solution of A s = b through a Householder QR of A."""
    Q, Rf = np.linalg.qr(A, mode="reduced")
    return np.linalg.solve(Rf, Q.T @ b)


def nnls(A, b, max_outer=None):
    """Lawson-Hanson NNLS.  Returns (x, resid2, info).

    Passive set P starts empty, x = 0.  Outer loop: w = A^T (b - A x); stop when
    every index outside P has w_j <= tol; otherwise move the index with the
    largest w_j (ties -> smallest index) into P.  Inner loop: solve the
    unconstrained problem on P; if some component is <= 0, step from x toward
    that solution as far as feasibility allows, move the indices that hit zero
    out of P (at least the one that limits the step, so the inner loop ends
    within |P| rounds), and repeat.  info = 1 when the outer-iteration cap
    (3 r) is hit.
    """
    A = np.asarray(A, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    p, r = A.shape
    if max_outer is None:
        max_outer = 3 * r
    eps = np.finfo(np.float64).eps
    tol = 10.0 * eps * np.abs(A).sum(axis=0).max(initial=0.0) * max(p, r)
    x = np.zeros(r)
    P = np.zeros(r, dtype=bool)
    info = 0
    outer = 0
    w = A.T @ (b - A @ x)
    while (~P).any():
        cand = np.where(~P, w, -np.inf)
        t = int(np.argmax(cand))
        if cand[t] <= tol:
            break
        if outer >= max_outer:
            info = 1
            break
        outer += 1
        P[t] = True
        while True:
            s = np.zeros(r)
            idx = np.flatnonzero(P)
            s[idx] = _ls(A[:, idx], b)
            if (s[idx] > 0).all():
                x = s
                break
            # step length: the largest alpha keeping x + alpha (s - x) >= 0 on
            # the indices whose unconstrained value is <= 0; an index already
            # at zero (x_u = 0, e.g. the one that just entered) allows no step
            bad = idx[s[idx] <= 0]
            if len(bad) == 0:                # NaN in the subproblem: no finite step
                info = 1
                break
            xb = x[bad]
            pos = xb > 0
            ratios = np.zeros(len(bad))
            ratios[pos] = xb[pos] / (xb[pos] - s[bad][pos])
            k = int(np.argmin(ratios))
            x = x + ratios[k] * (s - x)
            x[bad[k]] = 0.0                  # the index that limits the step is at its bound
            drop = P & (x <= tol)
            x[drop] = 0.0
            P &= ~drop
            if not P.any():
                break
        w = A.T @ (b - A @ x)
    resid2 = float(np.sum((A @ x - b) ** 2))
    return x, resid2, info


def nnls_matrix(M, K, cols=None):
    """H (r x n) with H(:, i) = NNLS(M(:, K), M(:, i)) for every column i.

    Returns (H, resid2 per column, info per column).
    """
    M = np.asarray(M, dtype=np.float64)
    K = list(K)
    A = M[:, K]
    n = M.shape[1]
    cols = range(n) if cols is None else cols
    H = np.zeros((len(K), n))
    res = np.zeros(n)
    inf = np.zeros(n, dtype=np.int32)
    for i in cols:
        H[:, i], res[i], inf[i] = nnls(A, M[:, i])
    return H, res, inf


def kkt_violation(A, b, x):
    """Largest violation of the NNLS optimality conditions, relative to
    ||A||_1 ||b||: x >= 0, w = A^T (b - A x) <= 0 where x = 0, w = 0 where x > 0."""
    A = np.asarray(A, dtype=np.float64)
    w = A.T @ (b - A @ x)
    scale = max(np.abs(A).sum(axis=0).max(initial=0.0) * max(np.linalg.norm(b), 1e-300), 1e-300)
    viol = max(0.0, -float(x.min(initial=0.0)))
    pos = x > 0
    if pos.any():
        viol = max(viol, float(np.abs(w[pos]).max()) / scale)
    if (~pos).any():
        viol = max(viol, float(max(0.0, w[~pos].max())) / scale)
    return viol
