"""The oracle's pins are strong enough: a plausible mistake planted in a copy of
an oracle module (a dropped term, a wrong sign, a wrong index, a transposed
operand) makes at least one pin fail.  Mutations are applied to the source
text on the CPU; the real oracle is untouched."""

import importlib
import inspect
import types

import numpy as np
import pytest
import scipy.optimize


def mutant(modname, old, new):
    src = inspect.getsource(importlib.import_module(f"oracle.{modname}"))
    assert old in src, f"pattern not found in oracle.{modname}: {old!r}"
    mod = types.ModuleType(f"oracle._mutant_{modname}")
    mod.__package__ = "oracle"
    exec(compile(src.replace(old, new, 1), f"<mutant of oracle.{modname}>", "exec"), mod.__dict__)
    return mod


def _rng(k):
    return np.random.default_rng([77, k])


def tsqr_pins_pass(t):
    """A subset of the R pins: LAPACK on a tiny input, Gram identity, tree
    invariance with an odd leaf count, Kronecker closed form, l1 sums."""
    A = _rng(1).standard_normal((30, 5))
    lap = np.linalg.qr(A, mode="r")
    lap[np.diag(lap) < 0, :] *= -1
    ok = np.abs(t.tsqr_r_final(A, leaf_rows=30) - lap).max() <= 1e-13 * np.abs(lap).max()
    X = _rng(2).uniform(size=(700, 6)) - 0.3
    R = t.tsqr_r_final(X, leaf_rows=100)       # 7 leaves: odd counts at two levels
    ok &= np.linalg.norm(R.T @ R - X.T @ X) / np.linalg.norm(X) ** 2 <= 1e-14
    ok &= bool(np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) >= 0))
    B = _rng(3).lognormal(size=(20, 3))
    RB = np.linalg.qr(B, mode="r")
    RB[np.diag(RB) < 0, :] *= -1
    ok &= np.abs(t.tsqr_r_final(np.kron(B, B), leaf_rows=64) - np.kron(RB, RB)).max() <= 1e-12 * np.abs(RB).max() ** 2
    d, s2, g = t.reference_sums(X, chunk=64)
    ok &= np.allclose(d, np.abs(X).sum(0), rtol=1e-13) and np.allclose(g, X.T @ X, rtol=1e-13)
    return bool(ok)


@pytest.mark.parametrize("old,new", [
    ("A[j:, j + 1:] -= tau * np.outer(v, w)", "A[j:, j + 1:] -= np.outer(v, w)"),   # dropped tau
    ("v[0] = 1.0", "v[0] = v[0]"),                                                 # wrong v head
    ("sigma = np.linalg.norm(x[1:])", "sigma = np.linalg.norm(x[2:])"),            # wrong index
    ("w = v @ A[j:, j + 1:]", "w = v @ A[j:, j:-1]"),                              # shifted columns
    ("            nxt.append(level[-1])\n", "            pass\n"),                 # odd node dropped
    ("R[neg, :] = -R[neg, :]", "R[:, neg] = -R[:, neg]"),                          # transposed flip
    ("s1 += np.abs(C).sum(axis=0)", "s1 += C.sum(axis=0)"),                        # abs dropped
    ("g += (C.T @ C)", "g += (C @ C.T)[:n, :n]"),                                  # transposed operand
])
def test_tsqr_mutants_are_caught(old, new):
    from oracle import tsqr
    assert tsqr_pins_pass(tsqr)
    assert not tsqr_pins_pass(mutant("tsqr", old, new))


def nnls_pins_pass(nn):
    ok = True
    for s in range(60):               # correlated columns: the backtracking branch runs
        rng = np.random.default_rng([78, s])
        k = 3 + s % 6
        A = rng.uniform(size=(12, k)) + 0.5
        b = A @ rng.standard_normal(k) + 0.1 * rng.standard_normal(12)
        x, _, _ = nn.nnls(A, b)
        xs, _ = scipy.optimize.nnls(A, b)
        ok &= np.abs(x - xs).max() <= 1e-10 * max(1, np.abs(xs).max())
    return bool(ok)


@pytest.mark.parametrize("old,new", [
    ("        w = A.T @ (b - A @ x)\n    resid2", "        w = A.T @ (A @ x - b)\n    resid2"),  # wrong sign
    ("t = int(np.argmax(cand))", "t = int(np.argmin(cand))"),                       # wrong pick
    ("s[idx] = _ls(A[:, idx], b)", "s[idx] = _ls(A[:, idx], b)[::-1]"),             # permuted solve
    ("drop = P & (x <= tol)", "drop = P & (x > tol)"),                               # wrong set dropped
])
def test_nnls_mutants_are_caught(old, new):
    """(Changing the backtracking step length alone is not a mistake that shows
    in the output: the outer loop of Lawson-Hanson re-adds any index dropped
    too early, so such variants still return the unique minimiser.)"""
    from oracle import nnls
    assert nnls_pins_pass(nnls)
    assert not nnls_pins_pass(mutant("nnls", old, new))


def spa_pins_pass(sel):
    rng = _rng(20)
    n, r = 14, 5
    K = sorted(rng.choice(n, size=r, replace=False).tolist())
    H = 2.0 * rng.uniform(size=(r, n))          # as in Sec. 4: columns do not sum to one
    H[:, K] = np.eye(r)
    X = rng.uniform(size=(200, r)) @ H
    d = X.sum(0)
    Kx, _, _ = sel.spa(X, r, colscale=d)
    M = np.array([[3.0, 0.0, 2.0], [0.0, 1.0, 2.0]])
    K2, _, _ = sel.spa(M, 2)
    Y = np.array([[1.0, 5.0, -2.0, 5.0], [0.0, 0.0, 3.0, -1.0], [2.0, 1.0, 1.0, 0.5]])
    Kg, _, _ = sel.gp_select(Y, 3)
    return sorted(Kx) == K and K2 == [0, 2] and Kg == [2, 3, 0]


@pytest.mark.parametrize("old,new", [
    ("Z = Z - np.outer(u, u @ Z)", "Z = Z + np.outer(u, u @ Z)"),                   # wrong sign
    ("u = Z[:, j] / np.sqrt(s[j])", "u = Z[:, j] / s[j]"),                          # wrong normalisation
    ("Z = M / np.asarray(colscale, dtype=np.float64)[None, :]", "Z = M * np.asarray(colscale, dtype=np.float64)[None, :]"),
    ("counts[int(np.argmin(Yn[l]))] += 1", "counts[int(np.argmax(Yn[l]))] += 1"),   # min dropped
])
def test_select_mutants_are_caught(old, new):
    from oracle import select
    assert spa_pins_pass(select)
    assert not spa_pins_pass(mutant("select", old, new))


def philox_pins_pass(ph):
    from tests.test_oracle_philox_gp import _rocrand_rounds
    tup = [(1, 2, 3, 4, 5, 6), (0xDEADBEEF, 0, 7, 0xFFFFFFFF, 123, 456)]
    ref = _rocrand_rounds(tup)
    got = np.array([[int(w) for w in ph.philox4x32_10(*t)] for t in tup], dtype=np.uint64)
    return bool(np.array_equal(got, ref))


@pytest.mark.parametrize("old,new", [
    ("c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,", "c0, c1, c2, c3 = (lo1 ^ c1 ^ np.uint64(k0), hi1,"),
    ("k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF", "k1 = k1"),
    ("for rnd in range(10):", "for rnd in range(9):"),
])
def test_philox_mutants_are_caught(old, new):
    from oracle import philox
    assert philox_pins_pass(philox)
    assert not philox_pins_pass(mutant("philox", old, new))


def xray_pins_pass(sel):
    """Brute-force XRAY picks (tests.test_oracle_select_nnls) on a few small
    matrices, and the hand-checked 2 x 3 case."""
    from tests.test_oracle_select_nnls import _xray_brute
    ok = True
    for seed in range(4):
        rng = np.random.default_rng([302, seed])
        M = rng.uniform(size=(6, 9))
        M[:, 3] *= 2.0
        K, _ = sel.xray(M, 3)
        ok &= K == _xray_brute(M, 3)
    for seed in range(6):                # wide and short: later picks differ more
        rng = np.random.default_rng([303, seed])
        M = rng.uniform(size=(4, 8))
        M[:, 1] *= 2.0
        K, _ = sel.xray(M, 4)
        ok &= K == _xray_brute(M, 4)
    M = np.array([[2.0, 0.0, 1.0], [0.0, 1.0, 1.0]])
    ok &= sel.xray(M, 2)[0] == [0, 1]
    return bool(ok)


@pytest.mark.parametrize("old,new", [
    ("Res = M - M[:, K] @ H", "Res = M + M[:, K] @ H"),                              # wrong sign
    ("Res = M - M[:, K] @ H", "Res = M - M[:, K[:1]] @ H[:1]"),                       # only the first pick fitted
    ("Res = M - M[:, K] @ H", "Res = M"),                                             # residual never updated
    ("np.linalg.norm(Res.T @ M[:, j])", "np.linalg.norm(M.T @ Res[:, j])"),          # score operands swapped
    ("np.linalg.norm(Res.T @ M[:, j]) / norms[j]", "np.linalg.norm(Res.T @ M[:, j])"),  # normalisation dropped
])
def test_xray_mutants_are_caught(old, new):
    from oracle import select
    assert xray_pins_pass(select)
    assert not xray_pins_pass(mutant("select", old, new))
