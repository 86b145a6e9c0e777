"""GPU parity of the one-pass state (tsnmf_onepass_*), through the C ABI: a
matrix pushed as consecutive row blocks, from device or host memory, gives
the R factor, the l1 column sums and G^T X of the whole matrix (Sec. 3.3 and
Sec. 3.5: one pass gives all three; Sec. 4 and Sec. 5.1 read matrices larger
than memory once, in splits).

Bars: R against the FP64 oracle of the whole matrix with the TSQR tests'
bounds (Gram error 1e-6 / element error 2e-5 for FP32 row blocks, 1e-12 /
1e-10 for FP64); the merge of the running R with each block's R is one more
FP64 tree node, so the bounds do not change.  Column sums: FP64 sums of the
blocks' sums.  G^T X: entry by entry within the projection tests' bound (the
rows one FP32 accumulator sums are fewer in a block than in the whole
matrix, so the whole matrix's bound holds).  Host input, pinned or pageable,
is bit-identical to device pushes of the same blocks, and a state saved and
loaded in the middle of a pass ends bit-identical to an uninterrupted one.
"""

import ctypes

import numpy as np
import pytest
import torch

from paper_1402_6964_amd import synth
from test_gpu_gp import Sums, all_groups
from test_gpu_tsqr import _check_against_oracle

pytestmark = pytest.mark.gpu


def _np(t):
    return t.cpu().numpy()


def _bounds(m, cuts):
    edges = [0] + list(cuts) + [m]
    return list(zip(edges[:-1], edges[1:]))


def test_device_blocks_match_oracle(lib):
    """30,011 x 25 FP32 in ragged blocks (one of a single row) with k = 16."""
    m, n, k, seed = 30_011, 25, 16, 20140227
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=41, dist="lognormal")
    Xd = X.cuda()
    op = lib.OnePass(n, k=k, seed=seed)
    for a, b in _bounds(m, [10_000, 10_001, 10_008]):
        op.push(Xd[a:b])
    R, cs, Y = op.result()
    torch.cuda.synchronize()
    assert op.rows == m
    _check_against_oracle(_np(R), _np(cs), X.numpy(), 1e-6, 2e-5, 1e-6, norm_tol=1e-5)
    s = Sums(X.numpy(), seed, cols=all_groups(k))
    ratio = np.abs(_np(Y).astype(np.float64) - s.Y) / s.bound_f32()
    print(f"G^T X: max error / bound = {ratio.max():.3f}")
    assert ratio.max() <= 1.0
    op.close()


def test_wide_blocks_match_oracle(lib):
    """200 columns (the wide leaf and the FP64 merge of 400 x 200 stacks)."""
    m, n = 6_001, 200
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=42, dist="lognormal")
    op = lib.OnePass(n)
    for a, b in _bounds(m, [3_000]):
        op.push(X[a:b].cuda())
    R, cs, _ = op.result()
    torch.cuda.synchronize()
    _check_against_oracle(_np(R), _np(cs), X.numpy(), 1e-6, 5e-5, 1e-6, norm_tol=1e-5)


def test_fp64_column_major_blocks(lib):
    """FP64 column-major: each block is a row range of the column-major matrix
    (its leading dimension stays the full m)."""
    m, n = 100_003, 40
    Xt = synth.random_matrix(n, m, dtype=torch.float64, seed_tag=43, dist="lognormal")
    X = Xt.t()                                   # m x n, column-major view
    Xd = Xt.cuda().t()
    op = lib.OnePass(n, dtype=torch.float64, col_major=True)
    for a, b in _bounds(m, [1, 50_000, 99_999]):
        op.push(Xd[a:b])
    R, cs, _ = op.result()
    torch.cuda.synchronize()
    _check_against_oracle(_np(R), _np(cs), X.numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)


def test_host_input_equals_device_blocks(lib):
    """600,000 x 64 FP32 from pageable (numpy) and pinned host memory, k = 8:
    bit-identical to device pushes of the same blocks (block_rows rows each)."""
    m, n, k, seed = 600_000, 64, 8, 5
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=44, dist="uniform")
    ref = lib.OnePass(n, k=k, seed=seed)
    br = ref.block_rows
    assert br == (64 << 20) // (n * 4)
    Xd = X.cuda()
    for a in range(0, m, br):
        ref.push(Xd[a:min(m, a + br)])
    R0, cs0, Y0 = ref.result()
    outs = []
    for src in (X.numpy(), X.pin_memory()):
        op = lib.OnePass(n, k=k, seed=seed)
        op.push_host(src)
        outs.append(op.result())
        torch.cuda.synchronize()
        assert op.rows == m
        op.close()
    torch.cuda.synchronize()
    for R, cs, Y in outs:
        assert torch.equal(R, R0) and torch.equal(cs, cs0) and torch.equal(Y, Y0)
    _check_against_oracle(_np(R0), _np(cs0), X.numpy(), 1e-6, None, 1e-6, norm_tol=1e-5)


def test_host_input_with_row_stride(lib):
    """Host rows with a stride larger than n (a column slice of a wider
    array) are gathered row by row; same result as the contiguous copy."""
    m, n = 70_001, 12
    W = synth.random_matrix(m, 20, dtype=torch.float32, seed_tag=45).numpy()
    a = lib.OnePass(n)
    a.push_host(W[:, :n])
    b = lib.OnePass(n)
    b.push_host(np.ascontiguousarray(W[:, :n]))
    Ra, csa, _ = a.result()
    Rb, csb, _ = b.result()
    torch.cuda.synchronize()
    assert torch.equal(Ra, Rb) and torch.equal(csa, csb)


def test_save_load_resumes_exactly(lib):
    """Save after two blocks, restore into a fresh state, push the rest: the
    same bits as the uninterrupted pass.  A state of other parameters refuses
    the saved bytes."""
    m, n, k, seed = 40_000, 25, 8, 77
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=46).cuda()
    blocks = _bounds(m, [9_000, 20_000, 33_333])
    full = lib.OnePass(n, k=k, seed=seed)
    for a, b in blocks:
        full.push(X[a:b])
    R0, cs0, Y0 = full.result()
    first = lib.OnePass(n, k=k, seed=seed)
    for a, b in blocks[:2]:
        first.push(X[a:b])
    blob = first.save()
    first.close()
    second = lib.OnePass(n, k=k, seed=seed)
    second.load(blob)
    assert second.rows == 20_000
    for a, b in blocks[2:]:
        second.push(X[a:b])
    R1, cs1, Y1 = second.result()
    torch.cuda.synchronize()
    assert torch.equal(R0, R1) and torch.equal(cs0, cs1) and torch.equal(Y0, Y1)
    other = lib.OnePass(n, k=k, seed=seed + 1)
    buf = ctypes.create_string_buffer(blob, len(blob))
    assert lib.tsnmf_onepass_load(other.h, ctypes.addressof(buf), len(blob)) == -2
    assert lib.tsnmf_onepass_load(other.h, ctypes.addressof(buf), len(blob) - 1) == -3


def test_result_before_any_push_is_zero(lib):
    op = lib.OnePass(9, k=4, seed=1)
    R, cs, Y = op.result()
    torch.cuda.synchronize()
    assert op.rows == 0
    assert not R.any() and not cs.any() and not Y.any()


def test_argument_errors(lib):
    h = ctypes.c_void_p()
    assert lib.tsnmf_onepass_create(0, lib.F32, 0, 0, h) == -1
    assert lib.tsnmf_onepass_create(257, lib.F32, 0, 0, h) == -1
    assert lib.tsnmf_onepass_create(8, lib.BF16, 0, 0, h) == -2
    assert lib.tsnmf_onepass_create(8, lib.F32, 5, 0, h) == -3
    assert lib.tsnmf_onepass_create(8, lib.F32 | lib.COL_MAJOR, 8, 0, h) == -3
    assert lib.tsnmf_onepass_create(8, lib.F64, 8, 0, h) == -3
    op = lib.OnePass(8)
    X = torch.zeros((10, 8), dtype=torch.float32, device="cuda")
    assert lib.tsnmf_onepass_push(op.h, X, 0, 8) == -3
    assert lib.tsnmf_onepass_push(op.h, X, 10, 7) == -4
    assert lib.tsnmf_onepass_push(op.h, None, 10, 8) == -2
    assert lib.tsnmf_onepass_push(None, X, 10, 8) == -1
    R = torch.empty((8, 8), dtype=torch.float64, device="cuda")
    assert lib.tsnmf_onepass_result(op.h, None) == -2
    col = lib.OnePass(8, dtype=torch.float64, col_major=True)
    Xh = np.zeros((10, 8))
    assert lib.tsnmf_onepass_push_host(col.h, Xh, 10, 8) == 4      # TSNMF_ERR_UNSUPPORTED
    assert lib.tsnmf_onepass_result(op.h, R) == 0


def test_single_column_and_blocks_shorter_than_n(lib):
    """n = 1 (R is the column's 2-norm), and 40 columns pushed in blocks of
    fewer rows than columns."""
    x = synth.random_matrix(1_001, 1, dtype=torch.float64, seed_tag=47).cuda()
    op = lib.OnePass(1, dtype=torch.float64)
    for a, b in _bounds(1_001, [1, 500]):
        op.push(x[a:b])
    R, cs, _ = op.result()
    torch.cuda.synchronize()
    xh = x.cpu().numpy()
    assert abs(R.item() - np.linalg.norm(xh)) <= 1e-14 * np.linalg.norm(xh)
    assert abs(cs.item() - np.abs(xh).sum()) <= 1e-13 * np.abs(xh).sum()
    m, n = 200, 40
    X = synth.random_matrix(m, n, dtype=torch.float64, seed_tag=48, dist="lognormal")
    op = lib.OnePass(n, dtype=torch.float64)
    for a in range(0, m, 13):                    # 13-row blocks, 40 columns
        op.push(X[a:a + 13].cuda())
    R, cs, _ = op.result()
    torch.cuda.synchronize()
    _check_against_oracle(_np(R), _np(cs), X.numpy(), 1e-12, 1e-10, 1e-13, norm_tol=1e-12)
