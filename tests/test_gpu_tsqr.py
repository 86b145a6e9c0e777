"""GPU parity of tsnmf_tsqr_r (Sec. 3.1 R factor, Sec. 3.3 column sums) against
the CPU oracle, through the C ABI.

Tolerances (the accuracy targets of the path): ||R^T R - X^T X||_F / ||X||_F^2 <= 1e-6 for
FP32 row blocks and <= 1e-12 for the FP64 path; column 2-norm relative error
<= 1e-5 (FP32).  Element-wise R comparisons use inputs with full column rank
and moderate condition number, where R is unique and first-order perturbation
theory bounds the difference by a small multiple of cond * eps; the bound is
stated per test.  Column sums: FP32 data summed in FP32 within a block of at
most 512 rows (at most 8 additions per lane, then a 64-lane tree) and in FP64
across blocks: relative error <= 1e-6; FP64 data: <= 1e-13.
"""

import numpy as np
import pytest
import torch

from oracle import tsqr as otsqr
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu


def _rel_gram(R, X64):
    G = X64.T @ X64
    return np.linalg.norm(R.T @ R - G) / np.linalg.norm(X64) ** 2


def _run(lib, X, **kw):
    torch.cuda.synchronize()
    R, cs = lib.tsqr_r(X, **kw)
    torch.cuda.synchronize()
    return R.cpu().numpy(), (cs.cpu().numpy() if cs is not None else None)


def _check_against_oracle(Rg, csg, Xh, gram_tol, elem_tol, cs_tol, norm_tol=None):
    X64 = np.asarray(Xh, dtype=np.float64)
    assert np.all(np.tril(Rg, -1) == 0.0), "strict lower triangle must be exactly zero"
    assert np.all(np.diag(Rg) >= 0.0), "diag(R) >= 0"
    g = _rel_gram(Rg, X64)
    assert g <= gram_tol, f"gram error {g:.3e} > {gram_tol:.1e}"
    if norm_tol is not None:
        cn = np.linalg.norm(X64, axis=0)
        nz = cn > 0
        rel = np.abs(np.linalg.norm(Rg, axis=0)[nz] - cn[nz]) / cn[nz]
        assert rel.max(initial=0.0) <= norm_tol, f"column-norm error {rel.max():.3e}"
    if elem_tol is not None:
        Ro = otsqr.tsqr_r_final(X64, leaf_rows=4096)
        err = np.abs(Rg - Ro).max() / np.abs(Ro).max()
        assert err <= elem_tol, f"R element error {err:.3e} > {elem_tol:.1e}"
    if csg is not None:
        d = np.abs(X64).sum(axis=0)
        nz = d > 0
        rel = np.abs(csg[nz] - d[nz]) / d[nz]
        assert rel.max(initial=0.0) <= cs_tol, f"colsum error {rel.max():.3e}"
        assert np.all(csg[~nz] == 0.0)


@pytest.mark.parametrize("n", [1, 2, 3, 7, 8, 16, 20, 25, 31, 32])
def test_fp32_rowmajor_contiguous(lib, n):
    """Staged row-major path: several blocks per slab, many slabs, ragged tail."""
    m = 200_003
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=1, dist="uniform")
    Rg, csg = _run(lib, X.cuda())
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("n", [5, 25])
def test_fp32_rowmajor_strided(lib, n):
    """Row-major with ld > n (direct loads)."""
    m = 70_001
    big = synth.random_matrix(m, n + 3, dtype=torch.float32, seed_tag=2, dist="lognormal")
    X = big[:, 1:n + 1]
    Rg, csg = _run(lib, big.cuda()[:, 1:n + 1])
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("n", [4, 20, 32])
def test_fp32_colmajor(lib, n):
    m = 150_007
    Xt = synth.random_matrix(n, m, dtype=torch.float32, seed_tag=3, dist="uniform")  # (n, m) contiguous
    X = Xt.t()
    Rg, csg = _run(lib, Xt.cuda().t())
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("n", [1, 6, 20, 32])
def test_fp64_rowmajor(lib, n):
    m = 100_000
    X = synth.random_matrix(m, n, dtype=torch.float64, seed_tag=4, dist="uniform")
    Rg, csg = _run(lib, X.cuda())
    _check_against_oracle(Rg, csg, X.numpy(), 1e-12, 1e-11, 1e-13, norm_tol=1e-12)


def test_plain_fp64_config(lib):
    """The plain FP64 workload: 100,000 x 20, r = 10, 1,000-row leaves and a
    binary tree; R against the oracle run with the same leaves and tree."""
    d = synth.plain_fp64()
    X = d["X"]
    cfg = lib.TsqrConfig(leaf_rows=1000, tree_arity=2, rows_per_lane=0)
    Rg, csg = _run(lib, X.cuda(), config=cfg)
    X64 = X.numpy()
    Ro = otsqr.tsqr_r_final(X64, leaf_rows=1000)
    # near-separable: rank 10 + 1e-3 noise, so cond(R) ~ 1e4; FP64 rounding ~ 1e-16 * cond
    assert np.abs(Rg - Ro).max() / np.abs(Ro).max() <= 1e-10
    _, _, G = otsqr.reference_sums_exact(X64)
    assert np.linalg.norm(Rg.T @ Rg - G) / np.linalg.norm(X64) ** 2 <= 1e-12
    d1 = np.abs(X64).sum(axis=0)
    assert np.abs(csg - d1).max() / d1.max() <= 1e-13


@pytest.mark.parametrize("n,leaf,m,layout,arity", [
    (1, 1000, 100_003, "row", 0), (7, 777, 60_001, "padded", 2), (13, 1000, 255_999, "row", 0),
    (13, 1000, 256_001, "row", 0), (20, 1024, 200_000, "padded", 0), (20, 1000, 100_000, "col", 2),
    (32, 300, 50_000, "row", 2), (32, 1024, 1_000, "row", 0)])
def test_fp64_short_slabs(lib, n, leaf, m, layout, arity):
    """FP64 slabs of one to eight blocks (at most 1,024 rows), at most 256 of
    them: the eight waves of a workgroup factor each slab as one block.  257
    slabs, column-major input and single-block slabs take the one-wave leaf;
    every case against the oracle run with the same leaves, ragged last
    slabs included."""
    X, _ = _layout_view(None, m, n, layout, torch.float64, 700 + n)
    cfg = lib.TsqrConfig(leaf_rows=leaf, tree_arity=arity, rows_per_lane=0)
    Rg, csg = _run(lib, X, config=cfg)
    X64 = X.cpu().numpy().astype(np.float64)
    Ro = otsqr.tsqr_r_final(X64, leaf_rows=leaf)
    assert np.all(np.tril(Rg, -1) == 0.0) and np.all(np.diag(Rg) >= 0.0)
    assert np.abs(Rg - Ro).max() / np.abs(Ro).max() <= 1e-11
    assert _rel_gram(Rg, X64) <= 1e-12
    d = np.abs(X64).sum(axis=0)
    assert np.abs(csg - d).max() / d.max() <= 1e-13


def test_fp32_input_fp64_leaves(lib):
    """TSNMF_LEAF_F64: FP32 bytes widened exactly, FP64 throughout."""
    X = synth.random_matrix(90_001, 17, dtype=torch.float32, seed_tag=5, dist="lognormal")
    Rg, csg = _run(lib, X.cuda(), leaf_f64=True)
    _check_against_oracle(Rg, csg, X.numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


def test_configs_give_the_same_r(lib):
    """Tree invariance on the GPU: leaf heights / arities change only rounding."""
    X = synth.random_matrix(123_457, 12, dtype=torch.float32, seed_tag=6).cuda()
    R0, _ = _run(lib, X)
    for leaf, arity in [(256, 2), (1000, 0), (5000, 2), (64, 2), (123_457, 2), (256, 3), (512, 7),
                        (256, 64), (1000, 16)]:
        cfg = lib.TsqrConfig(leaf_rows=leaf, tree_arity=arity, rows_per_lane=0)
        R1, _ = _run(lib, X, config=cfg)
        assert np.abs(R1 - R0).max() / np.abs(R0).max() <= 1e-5


def test_deterministic(lib):
    X = synth.random_matrix(300_000, 25, dtype=torch.float32, seed_tag=7).cuda()
    R0, c0 = _run(lib, X)
    R1, c1 = _run(lib, X)
    assert np.array_equal(R0, R1) and np.array_equal(c0, c1)


@pytest.mark.parametrize("m,n", [(1, 1), (1, 5), (3, 8), (8, 8), (64, 32), (65, 3)])
def test_short_inputs(lib, m, n):
    """m < n and m <= one block: R is the factor of X padded with zero rows."""
    X = synth.random_matrix(m, n, dtype=torch.float64, seed_tag=8, dist="normal")
    Rg, csg = _run(lib, X.cuda())
    Ro = otsqr.tsqr_r_final(X.numpy(), leaf_rows=1000)
    assert np.abs(Rg - Ro).max() <= 1e-12 * max(1.0, np.abs(Ro).max())
    assert np.allclose(csg, np.abs(X.numpy()).sum(0), rtol=1e-14, atol=0)


def test_zero_column_and_zero_matrix(lib):
    X = synth.random_matrix(5000, 6, dtype=torch.float32, seed_tag=9)
    X[:, 3] = 0.0
    Rg, csg = _run(lib, X.cuda())
    assert np.all(Rg[:, 3] == 0.0) or np.abs(Rg[:, 3]).max() <= 1e-6 * np.abs(Rg).max()
    assert np.linalg.norm(Rg.T @ Rg - X.double().numpy().T @ X.double().numpy()) / np.linalg.norm(X.double().numpy()) ** 2 <= 1e-6
    assert csg[3] == 0.0
    Z = torch.zeros((1000, 4), dtype=torch.float32, device="cuda")
    Rz, cz = _run(lib, Z)
    assert np.all(Rz == 0.0) and np.all(cz == 0.0)


def test_nan_propagates(lib):
    X = synth.random_matrix(10_000, 5, dtype=torch.float32, seed_tag=10)
    X[777, 2] = float("nan")
    Rg, csg = _run(lib, X.cuda())
    assert np.isnan(csg[2]) and np.isnan(Rg).any()


def test_kronecker_full_size(lib):
    """Flow-cytometry shape at full size (3162^2 x 25 ~ 1e7 rows, FP32, the
    Sec. 5.2 construction X = A (x) A): R = R_A (x) R_A and colsum = d_A (x) d_A,
    both from the oracle on the 3162 x 5 factor alone."""
    d = synth.flow_kron(p=3162, q=5, device="cuda")
    Rg, csg = _run(lib, d["X"])
    A = d["A"].astype(np.float64)
    RA = otsqr.tsqr_r_final(A, leaf_rows=1000)
    ref = np.kron(RA, RA)
    # entries of X are FP32-rounded products (relative 6e-8) and the leaves are FP32
    assert np.abs(Rg - ref).max() / np.abs(ref).max() <= 2e-5
    dA = np.abs(A).sum(0)
    assert np.abs(csg - np.kron(dA, dA)).max() / np.kron(dA, dA).max() <= 1e-6


@pytest.mark.parametrize("n,dt", [(25, torch.float32), (2, torch.float32), (40, torch.float32), (20, torch.float64)])
def test_more_than_2_31_elements(lib, n, dt):
    """Row-major inputs with more than 2^31 elements (64-bit row offsets in the
    staged and wide leaves): t stacked copies of a block A give R = sqrt(t) R_A
    and colsum = t d_A, with R_A and d_A from the oracle on A alone."""
    elems = (1 << 31) + (1 << 27)
    mA = 50_000
    t = -(-elems // (mA * n))
    A = synth.random_matrix(mA, n, dtype=dt, seed_tag=27, dist="lognormal")
    X = A.cuda().repeat(t, 1)
    assert X.numel() > (1 << 31)
    Rg, csg = _run(lib, X)
    del X
    torch.cuda.empty_cache()
    Ah = A.numpy().astype(np.float64)
    ref = np.sqrt(t) * otsqr.tsqr_r_final(Ah, leaf_rows=5000)
    f32 = dt == torch.float32
    gram = np.linalg.norm(Rg.T @ Rg - ref.T @ ref) / np.linalg.norm(ref) ** 2
    assert gram <= (1e-6 if f32 else 1e-12), f"gram error {gram:.3e}"
    cn = np.linalg.norm(ref, axis=0)
    assert np.max(np.abs(np.linalg.norm(Rg, axis=0) - cn) / cn) <= (1e-5 if f32 else 1e-12)
    dA = np.abs(Ah).sum(0)
    assert np.max(np.abs(csg - t * dA) / (t * dA)) <= (1e-6 if f32 else 1e-13)


def test_invalid_arguments(lib):
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    R = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    assert lib.tsnmf_tsqr_r(None, 10, 4, 4, lib.F32, R) == -1
    assert lib.tsnmf_tsqr_r(X, 0, 4, 4, lib.F32, R) == -2
    assert lib.tsnmf_tsqr_r(X, 10, 0, 4, lib.F32, R) == -3
    assert lib.tsnmf_tsqr_r(X, 10, 4, 3, lib.F32, R) == -4
    assert lib.tsnmf_tsqr_r(X, 10, 4, 9, lib.F32 | lib.COL_MAJOR, R) == -4
    assert lib.tsnmf_tsqr_r(X, 10, 4, 4, lib.BF16, R) == -5
    assert lib.tsnmf_tsqr_r(X, 10, 4, 4, lib.F32, None) == -6
    assert lib.tsnmf_tsqr_r(X, 10, 300, 300, lib.F32, R) == 4
    for arity in (1, 65, -2):
        bad = lib.TsqrConfig(leaf_rows=0, tree_arity=arity, rows_per_lane=0)
        assert lib.tsnmf_tsqr_r_ex(X, 10, 4, 4, lib.F32, R, None, bad) == -8


# ---- wide factors (33..128 columns) ------------------------------------------------

@pytest.mark.parametrize("n", [33, 48, 64, 100, 128])
def test_wide_fp32_rowmajor(lib, n):
    m = 60_017
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=20, dist="uniform")
    Rg, csg = _run(lib, X.cuda())
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6, 5e-5, 1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("n", [40, 64, 128])
def test_wide_fp32_colmajor(lib, n):
    m = 80_021
    Xt = synth.random_matrix(n, m, dtype=torch.float32, seed_tag=21, dist="lognormal")
    Rg, csg = _run(lib, Xt.cuda().t())
    _check_against_oracle(Rg, csg, Xt.t().numpy(), 1e-6, 5e-5, 1e-6, norm_tol=1e-5)


@pytest.mark.parametrize("n", [64, 128])
def test_wide_fp64(lib, n):
    X = synth.random_matrix(40_000, n, dtype=torch.float64, seed_tag=22, dist="uniform")
    Rg, csg = _run(lib, X.cuda())
    _check_against_oracle(Rg, csg, X.numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


def test_wide_fp32_input_fp64_leaves(lib):
    X = synth.random_matrix(50_003, 96, dtype=torch.float32, seed_tag=23, dist="uniform")
    Rg, csg = _run(lib, X.cuda(), leaf_f64=True)
    _check_against_oracle(Rg, csg, X.numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


@pytest.mark.parametrize("n,dt", [(48, torch.float32), (100, torch.float32), (64, torch.float64), (90, torch.float64)])
def test_wide_rowmajor_strided(lib, n, dt):
    """A column window of a wider row-major array (ld = n + 7, offset 3)."""
    m = 30_011
    store = synth.random_matrix(m, n + 7, dtype=dt, seed_tag=25, dist="uniform")
    X = store[:, 3:3 + n]
    Rg, csg = _run(lib, store.cuda()[:, 3:3 + n])
    f32 = dt == torch.float32
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6 if f32 else 1e-12, 5e-5 if f32 else 1e-10,
                          1e-6 if f32 else 1e-13, norm_tol=1e-5 if f32 else 1e-12)


@pytest.mark.parametrize("n,dt", [(100, torch.float32), (70, torch.float64), (40, torch.float64)])
def test_wide_rowmajor_huge_stride(lib, n, dt):
    """Row stride so large (ld = 900,000) that a block's row offsets leave the
    32-bit range of a buffer resource: the wide leaf falls back to
    per-element 64-bit addresses."""
    m, ld = 2_500, 900_000
    X = synth.random_matrix(m, n, dtype=dt, seed_tag=28, dist="uniform")
    store = torch.zeros((m, ld), dtype=dt, device="cuda")
    store[:, :n] = X.cuda()
    Rg, csg = _run(lib, store[:, :n])
    del store
    torch.cuda.empty_cache()
    f32 = dt == torch.float32
    _check_against_oracle(Rg, csg, X.numpy(), 1e-6 if f32 else 1e-12, 5e-5 if f32 else 1e-10,
                          1e-6 if f32 else 1e-13, norm_tol=1e-5 if f32 else 1e-12)


@pytest.mark.parametrize("m,n", [(1, 33), (40, 64), (65, 70), (129, 128), (1000, 40)])
def test_wide_short_inputs(lib, m, n):
    """Fewer rows than one 64-row chunk, one chunk plus a ragged tail, and
    inputs shorter than the block: the rows past m enter as zeros."""
    for dt in (torch.float32, torch.float64):
        X = synth.random_matrix(m, n, dtype=dt, seed_tag=26, dist="uniform")
        Rg, csg = _run(lib, X.cuda())
        X64 = X.numpy().astype(np.float64)
        f32 = dt == torch.float32
        assert np.all(np.tril(Rg, -1) == 0.0)
        g = _rel_gram(Rg, X64)
        assert g <= (1e-6 if f32 else 1e-12), f"m={m} n={n} {dt}: gram error {g:.3e}"
        d = np.abs(X64).sum(axis=0)
        assert np.max(np.abs(csg - d) / d) <= (1e-6 if f32 else 1e-13)


def test_wide_tree_shapes(lib):
    """Leaf counts 1, 2, 3, 5 and 37 exercise odd nodes at several levels."""
    X = synth.random_matrix(30_000, 70, dtype=torch.float32, seed_tag=24).cuda()
    Xh = X.cpu().numpy()
    for leaf in [30_000, 15_000, 10_000, 6_000, 811]:
        cfg = lib.TsqrConfig(leaf_rows=leaf, tree_arity=0, rows_per_lane=0)
        Rg, csg = _run(lib, X, config=cfg)
        _check_against_oracle(Rg, csg, Xh, 1e-6, 5e-5, 1e-6)


def test_heat_transfer_tiled_full_size(lib):
    """Heat-transfer shape at full size: 50,000,000 x 64 FP32 column-major
    (12.8 GB) built as 1,000 copies of a 50,000 x 64 bump-sum block A, so that
    R = sqrt(1000) R_A with R_A from the oracle, and colsum = 1000 d_A."""
    blk = synth.heat_transfer(m=50_000, n=64, device="cuda")
    A = blk["X"]                                  # (50000, 64) column-major view
    t = 1000
    store = A.t().contiguous().repeat(1, t)       # (64, 5e7): column-major X with ld = m
    X = store.t()
    Rg, csg = _run(lib, X)
    del store, X
    torch.cuda.empty_cache()
    Ah = A.cpu().numpy().astype(np.float64)
    ref = np.sqrt(t) * otsqr.tsqr_r_final(Ah, leaf_rows=5000)
    gram = np.linalg.norm(Rg.T @ Rg - ref.T @ ref) / np.linalg.norm(ref) ** 2
    assert gram <= 1e-6
    cn = np.linalg.norm(ref, axis=0)
    assert np.max(np.abs(np.linalg.norm(Rg, axis=0) - cn) / cn) <= 1e-5
    dA = np.abs(Ah).sum(0)
    assert np.max(np.abs(csg - t * dA) / (t * dA)) <= 1e-6


@pytest.mark.parametrize("n", [1, 16, 25, 32])
def test_tree_group_sizes_match_oracle(lib, n):
    """Every tree group size (2 .. 64 nodes per pass, capped by the pass
    capacity), with passes that use 1, 2, 4 or all 8 waves, against the oracle."""
    X = synth.random_matrix(400_003, n, dtype=torch.float32, seed_tag=60 + n, dist="uniform")
    Xh = X.numpy()
    Xd = X.cuda()
    for arity in (2, 3, 5, 8, 13, 40, 64):
        cfg = lib.TsqrConfig(leaf_rows=1024, tree_arity=arity, rows_per_lane=0)
        Rg, csg = _run(lib, Xd, config=cfg)
        _check_against_oracle(Rg, csg, Xh, 1e-6, 2e-5, 1e-6, norm_tol=1e-5)


def test_profiling_modes(lib):
    """on = 1 times the leaf and the tree; on = 2 the leaf only."""
    X = synth.random_matrix(200_000, 25, dtype=torch.float32, seed_tag=70).cuda()
    for mode, tree_calls in ((1, 3), (2, 0)):
        lib.tsnmf_profile_query(0)
        lib.tsnmf_profile_query(1)
        lib.tsnmf_profile_enable(mode)
        for _ in range(3):
            lib.tsqr_r(X)
        lib.tsnmf_profile_enable(0)
        st0, ms0, c0 = lib.tsnmf_profile_query(0)
        st1, ms1, c1 = lib.tsnmf_profile_query(1)
        assert st0 == 0 and st1 == 0 and c0 == 3 and c1 == tree_calls and ms0 > 0.0


def _layout_view(store_rows, m, n, layout, dt, tag):
    """X (m x n) as row-major contiguous, column-major (ld = m) or row-major
    with a padded row stride (ld = n + 5, offset 2)."""
    if layout == "row":
        base = synth.random_matrix(m, n, dtype=dt, seed_tag=tag, dist="uniform").cuda()
        return base, base
    if layout == "col":
        base = synth.random_matrix(n, m, dtype=dt, seed_tag=tag, dist="uniform").cuda()
        return base.t(), base
    base = synth.random_matrix(m, n + 5, dtype=dt, seed_tag=tag, dist="uniform").cuda()
    return base[:, 2:2 + n], base


@pytest.mark.parametrize("layout", ["row", "col", "padded"])
@pytest.mark.parametrize("n", [20, 96])
@pytest.mark.parametrize("path", ["f64", "f32_leaf_f64"])
def test_fp64_paths_every_layout(lib, path, n, layout):
    """The FP64 leaf kernels (FP64 input, and FP32 input with TSNMF_LEAF_F64)
    on every layout: row-major contiguous, column-major and a padded row
    stride, small and wide widths, at the FP64 tolerances."""
    dt = torch.float64 if path == "f64" else torch.float32
    X, _ = _layout_view(None, 60_007, n, layout, dt, 400 + n)
    Rg, csg = _run(lib, X, leaf_f64=(path != "f64"))
    _check_against_oracle(Rg, csg, X.cpu().numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


def test_graph_capture_single_calls_survive_growth(lib):
    """tsnmf_tsqr_r and tsnmf_gauss_proj captured into one graph after
    tsnmf_reserve; every replay (with eager work and synchronisation between
    replays, and new data in the same input buffer) matches an eager call.  A
    larger uncaptured call in between grows the workspace: the captured graph
    still names the old buffer, which the library keeps (not frees), so later
    replays stay correct."""
    m, n, k = 300_001, 25, 64
    lib.reserve(m, n, k)
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=410).cuda()
    R = torch.empty((n, n), dtype=torch.float64, device="cuda")
    cs = torch.empty(n, dtype=torch.float64, device="cuda")
    Y = torch.empty((n, k), dtype=torch.float32, device="cuda")
    s = torch.cuda.Stream()

    def calls(stream):
        assert lib.tsnmf_tsqr_r(X, m, n, n, lib.F32, R, cs, stream) == 0
        assert lib.tsnmf_gauss_proj(X, m, n, n, lib.F32 | lib.GP_SIMD_F32, k, 5, 0, Y, None, stream) == 0

    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=s):
        calls(s.cuda_stream)
    torch.cuda.synchronize()

    def eager():
        Re = torch.empty_like(R)
        ce = torch.empty_like(cs)
        Ye = torch.empty_like(Y)
        st = torch.cuda.current_stream().cuda_stream
        assert lib.tsnmf_tsqr_r(X, m, n, n, lib.F32, Re, ce, st) == 0
        assert lib.tsnmf_gauss_proj(X, m, n, n, lib.F32 | lib.GP_SIMD_F32, k, 5, 0, Ye, None, st) == 0
        torch.cuda.synchronize()
        return Re.cpu(), ce.cpu(), Ye.cpu()

    for rep in range(4):
        if rep == 2:
            # grow the workspace from outside the graph
            big = synth.random_matrix(2_000_000, 128, dtype=torch.float32, seed_tag=411).cuda()
            Rb, _ = lib.tsqr_r(big)
            torch.cuda.synchronize()
            del big
        X.mul_(1.5)                       # new data in the captured input buffer
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        Rg, cg, Yg = R.cpu(), cs.cpu(), Y.cpu()
        Re, ce, Ye = eager()
        assert torch.equal(Rg, Re) and torch.equal(cg, ce) and torch.equal(Yg, Ye), f"replay {rep}"
    _check_against_oracle(R.t().cpu().numpy(), cs.cpu().numpy(), X.cpu().numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)
    del g
    assert lib.tsnmf_workspace_release() == 0


@pytest.mark.parametrize("n,layout,dt", [(129, "row", torch.float32), (200, "col", torch.float32),
                                         (256, "row", torch.float32), (256, "padded", torch.float32),
                                         (160, "row", torch.float64), (256, "col", torch.float64)])
def test_widest_paths(lib, n, layout, dt):
    """129..256 columns (8 waves x 32 columns, R of each workgroup in global
    memory): R against the oracle at the precision's tolerances, for FP32 and
    FP64 input, row-major, column-major and a padded row stride."""
    m = 50_011
    X, _ = _layout_view(None, m, n, layout, dt, 500 + n)
    Rg, csg = _run(lib, X)
    if dt == torch.float32:
        _check_against_oracle(Rg, csg, X.cpu().numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)
    else:
        _check_against_oracle(Rg, csg, X.cpu().numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


def test_widest_fp32_input_fp64_leaves_and_short(lib):
    X = synth.random_matrix(30_007, 180, dtype=torch.float32, seed_tag=510, dist="uniform").cuda()
    Rg, csg = _run(lib, X, leaf_f64=True)
    _check_against_oracle(Rg, csg, X.cpu().numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)
    for m in (1, 100, 256, 257):
        Xs = synth.random_matrix(m, 256, dtype=torch.float32, seed_tag=511, dist="uniform").cuda()
        Rg, csg = _run(lib, Xs)
        X64 = Xs.cpu().numpy().astype(np.float64)
        assert np.all(np.tril(Rg, -1) == 0.0) and np.all(np.diag(Rg) >= 0.0)
        assert _rel_gram(Rg, X64) <= 1e-6


@pytest.mark.parametrize("n,layout,leaf_rows", [(33, "col", 0), (40, "row", 2048), (48, "col", 2048),
                                                (49, "row", 0), (64, "col", 2048), (64, "row", 1536),
                                                (57, "padded", 2048), (64, "col", 777)])
def test_wy_leaf_matches_oracle_and_unblocked(lib, n, layout, leaf_rows):
    """The blocked compact-WY leaf (FP32 row blocks, 33..64 columns, 16-column
    panels with the trailing update on the matrix cores): R against the oracle,
    and against the unblocked leaf on the same input (both compute the same R
    up to rounding).  Slabs of several 512-row blocks, a slab height that is
    not a whole number of blocks, and ragged last blocks."""
    m = 100_003
    X, _ = _layout_view(None, m, n, layout, torch.float32, 600 + n)
    cfg = lib.TsqrConfig(leaf_rows=leaf_rows, tree_arity=0, rows_per_lane=0, wy_panel=16)
    Rg, csg = _run(lib, X, config=cfg)
    _check_against_oracle(Rg, csg, X.cpu().numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)
    cfg1 = lib.TsqrConfig(leaf_rows=leaf_rows, tree_arity=0, rows_per_lane=0, wy_panel=1)
    Ru, _ = _run(lib, X, config=cfg1)
    assert np.abs(Rg - Ru).max() <= 2e-5 * np.abs(Ru).max()


@pytest.mark.parametrize("m,n", [(1, 40), (10, 64), (63, 64), (64, 33), (511, 48), (513, 64)])
def test_wy_leaf_short_inputs(lib, m, n):
    X = synth.random_matrix(n, m, dtype=torch.float32, seed_tag=610, dist="uniform").cuda().t()
    Rg, csg = _run(lib, X, config=lib.TsqrConfig(leaf_rows=0, tree_arity=0, rows_per_lane=0, wy_panel=16))
    X64 = X.cpu().numpy().astype(np.float64)
    assert np.all(np.tril(Rg, -1) == 0.0) and np.all(np.diag(Rg) >= 0.0)
    assert _rel_gram(Rg, X64) <= 1e-6
    d = np.abs(X64).sum(0)
    assert np.max(np.abs(csg - d) / d) <= 1e-6


def test_wy_panel_argument(lib):
    X = torch.zeros((100, 40), dtype=torch.float32, device="cuda")
    R = torch.empty((40, 40), dtype=torch.float64, device="cuda")
    for bad in (2, 8, 32, -1):
        cfg = lib.TsqrConfig(leaf_rows=0, tree_arity=0, rows_per_lane=0, wy_panel=bad)
        assert lib.tsnmf_tsqr_r_ex(X, 100, 40, 40, lib.F32, R, None, cfg) == -8


@pytest.mark.parametrize("p,q", [(3162, 5), (2000, 4), (1500, 3), (777, 2), (1000, 1)])
def test_kron_matches_explicit_bit_for_bit(lib, p, q):
    """tsnmf_tsqr_r_kron forms each row of X = A (x) A from two rows of A, with
    the plan of the explicit FP32 X: R and the column sums equal those of
    tsnmf_tsqr_r on the explicit matrix bit for bit, and R = R_A (x) R_A to
    FP32 accuracy (the products are rounded to FP32 once, as in X)."""
    A = torch.from_numpy(synth.kron_factor(p, 5)[:, :q].copy()).cuda()
    X = torch.kron(A, A).contiguous()
    Re, ce = lib.tsqr_r(X)
    Rk, ck = lib.tsqr_r_kron(A)
    torch.cuda.synchronize()
    assert torch.equal(Re, Rk) and torch.equal(ce, ck)
    Ah = A.cpu().numpy().astype(np.float64)
    RA = np.linalg.qr(Ah, mode="r")
    RA[np.diag(RA) < 0, :] *= -1
    Rkh = Rk.cpu().numpy()
    assert np.abs(Rkh - np.kron(RA, RA)).max() <= 2e-5 * np.abs(RA).max() ** 2
    dA = np.abs(Ah).sum(0)
    assert np.max(np.abs(ck.cpu().numpy() - np.kron(dA, dA)) / np.kron(dA, dA)) <= 1e-6


@pytest.mark.timeout(300)
def test_kron_paper_flow_cytometry_size(lib):
    """The Sec. 5.2 size: A of 40,000 cells x 5 markers, X = A (x) A with
    1.6e9 rows x 25 columns (160 GB in FP32, never formed).  R against the
    closed form R_A (x) R_A and the Gram identity R^T R = (A^T A) (x) (A^T A),
    column sums against d_A (x) d_A."""
    A = torch.from_numpy(synth.kron_factor(40_000, 5)).cuda()
    Rk, ck = lib.tsqr_r_kron(A)
    torch.cuda.synchronize()
    Ah = A.cpu().numpy().astype(np.float64)
    RA = np.linalg.qr(Ah, mode="r")
    RA[np.diag(RA) < 0, :] *= -1
    R = Rk.cpu().numpy()
    assert np.all(np.tril(R, -1) == 0.0) and np.all(np.diag(R) >= 0.0)
    G = np.kron(Ah.T @ Ah, Ah.T @ Ah)
    assert np.linalg.norm(R.T @ R - G) / np.linalg.norm(G) <= 1e-6
    assert np.abs(R - np.kron(RA, RA)).max() <= 2e-5 * np.abs(RA).max() ** 2
    dA = np.abs(Ah).sum(0)
    assert np.max(np.abs(ck.cpu().numpy() - np.kron(dA, dA)) / np.kron(dA, dA)) <= 1e-6


def test_kron_argument_errors(lib):
    A = torch.ones((10, 5), dtype=torch.float32, device="cuda")
    R = torch.empty((25, 25), dtype=torch.float64, device="cuda")
    assert lib.tsnmf_tsqr_r_kron(None, 10, 5, 5, R) == -1
    assert lib.tsnmf_tsqr_r_kron(A, 0, 5, 5, R) == -2
    assert lib.tsnmf_tsqr_r_kron(A, 10, 6, 6, R) == -3
    assert lib.tsnmf_tsqr_r_kron(A, 10, 5, 4, R) == -4
    assert lib.tsnmf_tsqr_r_kron(A, 10, 5, 5, None) == -5
