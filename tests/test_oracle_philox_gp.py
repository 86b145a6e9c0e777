"""Pins for oracle.philox and oracle.gauss_proj (Sec. 2.3, Sec. 3.2 / Algorithm 1,
Sec. 3.3)."""

import os
import shutil
import subprocess
import tempfile

import numpy as np
import pytest

from oracle import gauss_proj, philox

HERE = os.path.dirname(os.path.abspath(__file__))


def _rocrand_rounds(inputs):
    """Evaluate rocRAND's Philox4x32-10 on (c0, c1, c2, c3, k0, k1) tuples."""
    inc = "/opt/rocm/include"
    if shutil.which("g++") is None or not os.path.exists(os.path.join(inc, "rocrand", "rocrand_philox4x32_10.h")):
        pytest.skip("rocRAND headers or g++ not available")
    with tempfile.TemporaryDirectory() as d:
        exe = os.path.join(d, "rounds")
        subprocess.run(["g++", "-O1", "-D__HIP_PLATFORM_AMD__", "-I", inc,
                        os.path.join(HERE, "philox_rocrand_rounds.cpp"), "-o", exe],
                       check=True, capture_output=True)
        txt = "\n".join(" ".join(str(int(v)) for v in t) for t in inputs) + "\n"
        out = subprocess.run([exe], input=txt, capture_output=True, text=True, check=True).stdout
    return np.array([[int(v) for v in line.split()] for line in out.strip().splitlines()], dtype=np.uint64)


def test_philox_matches_rocrand_block_function():
    """P13: the oracle's Philox4x32-10 equals rocRAND's on random and edge
    counters/keys (rocRAND is an independent implementation of the same
    published generator)."""
    rng = np.random.default_rng(5)
    tup = [(0, 0, 0, 0, 0, 0), (0xFFFFFFFF,) * 6, (1, 2, 3, 4, 5, 6)]
    tup += [tuple(int(v) for v in rng.integers(0, 2 ** 32, size=6, dtype=np.uint64)) for _ in range(200)]
    ref = _rocrand_rounds(tup)
    got = np.array([[int(w) for w in philox.philox4x32_10(t[0], t[1], t[2], t[3], t[4], t[5])] for t in tup],
                   dtype=np.uint64)
    assert np.array_equal(got, ref)


def test_philox_known_answers():
    """The published known-answer vectors of Philox4x32-10 (golden fixture)."""
    rows = []
    with open(os.path.join(HERE, "golden", "philox4x32_10_kat.txt")) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                rows.append([int(v, 16) for v in line.split()])
    assert len(rows) == 3
    for r in rows:
        got = [int(w) for w in philox.philox4x32_10(*r[:6])]
        assert got == r[6:], f"counter/key {r[:6]}"


def test_uniform_range_endpoints():
    u = philox.uniform_open0(np.array([0, 255, 256, 0xFFFFFFFF], dtype=np.uint64))
    assert u[0] == 2.0 ** -24 and u[1] == 2.0 ** -24 and u[2] == 2.0 ** -23 and u[3] == 1.0


def test_gaussian_moments():
    """N(0, 1) moments over 4e5 draws: mean 0, variance 1, kurtosis 3, and the
    four outputs of one counter are uncorrelated."""
    G = philox.gaussian_matrix(14026964, 0, 100_000, 4)
    x = G.ravel()
    se = 1.0 / np.sqrt(x.size)
    assert abs(x.mean()) < 5 * se
    assert abs(x.var() - 1.0) < 5 * np.sqrt(2.0) * se
    assert abs(np.mean(x ** 4) - 3.0) < 5 * np.sqrt(96.0) * se
    C = np.corrcoef(G.T)
    assert np.abs(C - np.eye(4)).max() < 5 / np.sqrt(G.shape[0])


def test_gaussian_matrix_is_a_function_of_row_and_column():
    """G(i, l) does not depend on how rows are grouped (Sec. 3.2's concern about
    per-processor sampling): blocks taken at different offsets agree."""
    A = philox.gaussian_matrix(7, 0, 300, 16)
    B = philox.gaussian_matrix(7, 100, 150, 16)
    assert np.array_equal(A[100:250], B)
    C = philox.gaussian_matrix(8, 0, 300, 16)
    assert not np.allclose(A, C)
    big = philox.gaussian_matrix(7, (1 << 32) + 5, 3, 8)
    assert np.all(np.isfinite(big)) and not np.allclose(big, A[5:8, :8])


def test_projection_is_linear_and_commutes_with_column_scaling():
    """P12 (Sec. 3.3): (G^T X) D^{-1} = G^T (X D^{-1}); the row-chunked
    accumulation (Algorithm 1's combiner) equals one product."""
    rng = np.random.default_rng(6)
    X = rng.lognormal(size=(3000, 6))
    d = X.sum(axis=0)
    Y = gauss_proj.gauss_proj(X, 32, 99, chunk=700)
    Yn = gauss_proj.gauss_proj(X / d, 32, 99, chunk=1000)
    assert np.abs(Y / d - Yn).max() <= 1e-12 * np.abs(Yn).max()
    G = philox.gaussian_matrix(99, 0, 3000, 32)
    assert np.abs(Y - G.T @ X).max() <= 1e-12 * np.abs(Y).max()
    Yg = gauss_proj.gauss_proj_group(X, 3, 99, chunk=512)
    assert np.abs(Yg - Y[12:16]).max() <= 1e-12 * np.abs(Y).max()


def test_projection_preserves_norms_on_average():
    """Johnson-Lindenstrauss sanity: E ||G^T x||^2 = k ||x||^2."""
    rng = np.random.default_rng(7)
    X = rng.uniform(size=(4000, 5))
    k = 256
    Y = gauss_proj.gauss_proj(X, k, 1234)
    ratio = np.sum(Y * Y, axis=0) / (k * np.sum(X * X, axis=0))
    assert np.all(np.abs(ratio - 1.0) < 5 * np.sqrt(2.0 / k))
