"""Pins for oracle.select, oracle.nnls and oracle.residual (Sec. 2.1-2.4, Sec. 4)."""

import numpy as np
import pytest
import scipy.optimize

from oracle import nnls, residual, select, tsqr


def _rng(*tag):
    return np.random.default_rng([23, *tag])


def _separable(m, n, r, seed, noise=0.0):
    """X = W H with H = I on a planted K and simplex columns elsewhere."""
    rng = _rng(seed)
    K = sorted(rng.choice(n, size=r, replace=False).tolist())
    H = rng.dirichlet(np.ones(r), size=n).T
    H[:, K] = np.eye(r)
    W = rng.uniform(size=(m, r))
    X = W @ H + noise * rng.uniform(size=(m, n))
    return X, K, H


# ---------------------------------------------------------------- NNLS ------

@pytest.mark.parametrize("seed", range(8))
def test_nnls_matches_scipy_and_kkt(seed):
    """P14: Lawson-Hanson agrees with scipy's NNLS and satisfies the KKT
    conditions (the minimiser is unique for a full-column-rank A)."""
    rng = _rng(100, seed)
    A = rng.standard_normal((12, 6))
    b = rng.standard_normal(12)
    x, res, info = nnls.nnls(A, b)
    xs, rs = scipy.optimize.nnls(A, b)
    assert info == 0
    assert np.abs(x - xs).max() <= 1e-10 * max(1.0, np.abs(xs).max())
    assert abs(np.sqrt(res) - rs) <= 1e-10 * max(1.0, rs)
    assert nnls.kkt_violation(A, b, x) <= 1e-12


def test_nnls_backtracking_cases_match_scipy():
    """Correlated columns with a mixed-sign unconstrained optimum: the inner
    (backtracking) loop of Lawson-Hanson runs in several of these cases."""
    ran = 0
    orig = nnls._ls
    for s in range(60):
        rng = np.random.default_rng([78, s])
        k = 3 + s % 6
        A = rng.uniform(size=(12, k)) + 0.5
        b = A @ rng.standard_normal(k) + 0.1 * rng.standard_normal(12)
        calls = [0]

        def counted(A_, b_):
            calls[0] += 1
            return orig(A_, b_)
        nnls._ls = counted
        try:
            x, _, info = nnls.nnls(A, b)
        finally:
            nnls._ls = orig
        ran += calls[0] > int((x > 0).sum())
        xs, _ = scipy.optimize.nnls(A, b)
        assert info == 0
        assert np.abs(x - xs).max() <= 1e-9 * max(1.0, np.abs(xs).max())
        assert nnls.kkt_violation(A, b, x) <= 1e-12
    assert ran >= 3


def test_nnls_exact_nonnegative_solution_recovered():
    rng = _rng(101)
    A = rng.uniform(size=(20, 5))
    y = np.array([0.0, 1.5, 0.0, 0.25, 3.0])
    x, res, info = nnls.nnls(A, A @ y)
    assert np.abs(x - y).max() <= 1e-12 and res <= 1e-24


def test_nnls_all_negative_correlation_gives_zero():
    A = np.eye(3)
    x, res, info = nnls.nnls(A, -np.ones(3))
    assert np.all(x == 0.0) and abs(res - 3.0) <= 1e-15


def test_nnls_reduced_space_equals_full_space():
    """P10 (Sec. 2.4): NNLS on R(:, K) vs R(:, i) equals NNLS on X."""
    X, K, _ = _separable(400, 12, 4, 102, noise=1e-2)
    R = tsqr.tsqr_r_final(X, leaf_rows=100)
    Hx, rx, _ = nnls.nnls_matrix(X, K)
    Hr, rr, _ = nnls.nnls_matrix(R, K)
    assert np.abs(Hx - Hr).max() <= 1e-10 * np.abs(Hx).max()
    assert np.allclose(rx, rr, rtol=1e-8, atol=1e-12 * np.sum(X * X))
    assert abs(residual.relative_residual(X, K, Hx) - residual.relative_residual(R, K, Hr)) <= 1e-12


# ---------------------------------------------------------------- SPA -------

@pytest.mark.parametrize("seed", range(5))
def test_spa_recovers_planted_columns(seed):
    """P7: exactly separable data with simplex H columns: SPA on X D^{-1} finds K,
    and SPA on R D^{-1} makes the same ordered picks (Sec. 2.2)."""
    X, K, _ = _separable(600, 15, 5, 200 + seed)
    d = np.abs(X).sum(axis=0)
    Kx, _, _ = select.spa(X, 5, colscale=d)
    R = tsqr.tsqr_r_final(X, leaf_rows=128)
    Kr, _, info = select.spa(R, 5, colscale=d)
    assert sorted(Kx) == K
    assert Kr == Kx and info == 5


def test_spa_brute_force_small():
    """First pick is the column of largest 2-norm; the second is the largest
    after removing the first direction (computed by hand on a 2 x 3 case)."""
    M = np.array([[3.0, 0.0, 2.0], [0.0, 1.0, 2.0]])
    K, scores, _ = select.spa(M, 2)
    assert K[0] == 0 and abs(scores[0] - 9.0) <= 1e-15
    # residual after projecting out e1: columns (0,0), (0,1), (0,2) -> pick 2
    assert K[1] == 2 and abs(scores[1] - 4.0) <= 1e-15


def test_spa_ties_go_to_smallest_index_and_stop_at_zero():
    M = np.array([[1.0, 1.0, 0.0], [0.0, 0.0, 0.0]])
    K, _, info = select.spa(M, 3)
    assert K == [0] and info == 1


# ---------------------------------------------------------------- XRAY ------

def test_xray_selects_planted_columns_on_separable_data():
    X, K, _ = _separable(300, 10, 3, 300)
    R = tsqr.tsqr_r_final(X, leaf_rows=64)
    Kx, info = select.xray(R, 4)
    assert set(K) <= set(Kx)


def test_xray_first_pick_brute_force():
    """t = 1: Res = M, score_j = ||M^T M_j|| / ||M_j||."""
    M = _rng(301).uniform(size=(5, 7))
    K, _ = select.xray(M, 1)
    scores = [np.linalg.norm(M.T @ M[:, j]) / np.linalg.norm(M[:, j]) for j in range(7)]
    assert K[0] == int(np.argmax(scores))


# ---------------------------------------------------------------- GP --------

def test_gp_select_brute_force():
    Y = np.array([[1.0, 5.0, -2.0, 5.0],
                  [0.0, 0.0, 3.0, -1.0],
                  [2.0, 1.0, 1.0, 0.5]])
    K, counts, info = select.gp_select(Y, 3)
    # row 0: min 2, max 1 (tie -> 1); row 1: min 3, max 2; row 2: min 3, max 0
    assert counts.tolist() == [1, 1, 2, 2]
    assert K == [2, 3, 0] and info == 3


def test_gp_select_uses_column_scaling():
    Y = np.array([[1.0, 4.0]])
    K, counts, _ = select.gp_select(Y, 2, colscale=np.array([1.0, 8.0]))
    assert counts.tolist() == [1, 1] and K == [0, 1]
    Y = np.array([[1.0, 4.0, 3.0]])
    K, _, _ = select.gp_select(Y, 1, colscale=np.array([1.0, 8.0, 1.0]))
    assert K == [1]      # scaled row (1, 0.5, 3): max 2, min 1 -> tie on count, index 1


# ---------------------------------------------------------------- residual --

def test_residual_zero_at_planted_rank_and_positive_below():
    """P8: the residual vanishes for exactly separable data at the planted K."""
    X, K, H = _separable(500, 12, 4, 400)
    R = tsqr.tsqr_r_final(X, leaf_rows=100)
    Hr, _, _ = nnls.nnls_matrix(R, K)
    assert residual.relative_residual(R, K, Hr) <= 1e-24
    assert np.abs(Hr - H).max() <= 1e-10          # P9: planted H recovered
    Hs, _, _ = nnls.nnls_matrix(R, K[:3])
    assert residual.relative_residual(R, K[:3], Hs) > 1e-6


@pytest.mark.timeout(60)
def test_nnls_entering_index_with_zero_value_terminates(monkeypatch):
    """Lawson-Hanson step length when the index that just entered gets an
    unconstrained value of exactly zero (possible in rounding): its ratio is
    0 (no step), not 0 / 0, and it leaves the passive set; the inner loop
    ends and the result still satisfies the optimality conditions."""
    from oracle import nnls as on
    rng = np.random.default_rng(3)
    A = rng.uniform(size=(30, 6))
    b = A @ np.array([0.5, 0.0, 1.0, 0.0, 0.2, 0.0]) + 0.01 * rng.uniform(size=30)
    real_ls = on._ls
    calls = {"n": 0}

    def ls_with_zero(Asub, rhs):
        s = real_ls(Asub, rhs)
        calls["n"] += 1
        if calls["n"] >= 2:            # from the second subproblem on: last component exactly 0
            s = s.copy()
            s[-1] = 0.0
        return s

    monkeypatch.setattr(on, "_ls", ls_with_zero)
    x, r2, info = on.nnls(A, b)
    assert np.all(np.isfinite(x)) and np.all(x >= 0)
    monkeypatch.setattr(on, "_ls", real_ls)
    xr, _, _ = on.nnls(A, b)
    assert on.kkt_violation(A, b, xr) <= 1e-10
    assert info in (0, 1)


def _xray_brute(M, picks):
    """Greedy XRAY picks written out independently of the oracle: the NNLS fit
    of each column on the chosen ones comes from scipy, and for a single chosen
    column from its closed form h = max(0, a^T b / a^T a)."""
    M = np.asarray(M, dtype=np.float64)
    n = M.shape[1]
    norms = np.linalg.norm(M, axis=0)
    K = []
    Res = M.copy()
    margins = []
    for _ in range(picks):
        sc = {j: np.linalg.norm(Res.T @ M[:, j]) / norms[j] for j in range(n) if j not in K and norms[j] > 0.0}
        order = sorted(sc, key=lambda j: (-sc[j], j))
        bj = order[0]
        if len(order) > 1:
            margins.append((sc[order[0]] - sc[order[1]]) / sc[order[0]])
        K.append(bj)
        A = M[:, K]
        if len(K) == 1:
            a = A[:, 0]
            H = np.maximum(0.0, (a @ M) / (a @ a))[None, :]
        else:
            H = np.stack([scipy.optimize.nnls(A, M[:, i])[0] for i in range(n)], axis=1)
        Res = M - A @ H
    _xray_brute.margins = margins
    return K


@pytest.mark.parametrize("seed", range(6))
def test_xray_later_picks_brute_force(seed):
    """Picks 2 and 3 of greedy XRAY (Sec. 2.1): after each pick the residual is
    M - M(:, K) H with H the nonnegative fit on the chosen columns.  Checked
    against a brute-force restatement whose fits come from the closed form for
    one column and from scipy's NNLS for two; the score margins are asserted so
    the comparison is not decided by rounding."""
    rng = _rng(302, seed)
    M = rng.uniform(size=(6, 9))
    M[:, 3] *= 2.0                     # spread the first scores
    K, _ = select.xray(M, 3)
    Kb = _xray_brute(M, 3)
    assert min(_xray_brute.margins) > 1e-9
    assert K == Kb
    M = np.random.default_rng([303, seed]).uniform(size=(4, 8))
    M[:, 1] *= 2.0
    Kb = _xray_brute(M, 4)
    assert min(_xray_brute.margins) > 1e-9
    assert select.xray(M, 4)[0] == Kb


def test_xray_second_pick_by_hand():
    """A 2 x 3 case small enough to check by hand.  Columns a = (2, 0),
    b = (0, 1), c = (1, 1).  Pick 1: scores ||M^T x|| / ||x|| are
    a: ||(4, 0, 2)|| / 2 = sqrt(5), b: ||(0, 1, 1)|| = sqrt(2),
    c: ||(2, 1, 2)|| / sqrt(2) = 3 / sqrt(2) -> a (sqrt 5 > 2.12).
    Fit on a: h = max(0, a^T x / 4) = (1, 0, 1/2); Res = M - a h =
    [(0,0), (0,1), (0,1)].  Pick 2: b: ||Res^T b|| / 1 = ||(0, 1, 1)|| = sqrt 2,
    c: ||Res^T c|| / sqrt 2 = ||(0, 1, 1)|| / sqrt 2 = 1 -> b."""
    M = np.array([[2.0, 0.0, 1.0], [0.0, 1.0, 1.0]])
    K, info = select.xray(M, 2)
    assert K == [0, 1] and info == 2
