"""tsnmf_tsqr_r_noalloc (the allocation-free TSQR entry point) through the C
ABI: two calls in a row, the second on a smaller input, each compared with
tsnmf_tsqr_r on the same input (R and column sums within the FP32-leaf or FP64
tolerances) and with the oracle."""

import numpy as np
import pytest
import torch

from oracle import tsqr as otsqr
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu


def _both(lib, X, flags):
    m, n = X.shape
    lay, ld = lib._layout(X)
    flags |= lay
    outs = []
    for fn in (lib.tsnmf_tsqr_r_noalloc, lib.tsnmf_tsqr_r):
        R = torch.full((n, n), float("nan"), dtype=torch.float64, device="cuda")
        cs = torch.full((n,), float("nan"), dtype=torch.float64, device="cuda")
        assert fn(X, m, n, ld, flags, R, cs) == 0
        torch.cuda.synchronize()
        outs.append((R.t().cpu().numpy(), cs.cpu().numpy()))
    return outs


def _check(lib, X, flags, rtol, gram_tol):
    print(f"noalloc case: {tuple(X.shape)} flags {flags:#x}", flush=True)
    (Ra, ca), (Rb, cb) = _both(lib, X, flags)
    assert np.all(np.tril(Ra, -1) == 0.0) and np.all(np.diag(Ra) >= 0.0)
    scale = np.abs(Rb).max()
    assert np.abs(Ra - Rb).max() <= rtol * scale
    Xh = X.cpu().numpy().astype(np.float64)
    # the two calls may cut the rows into different slabs (the scratch array
    # bounds the leaves), so FP32 sums round differently: the FP32 bar
    d = np.abs(Xh).sum(axis=0)
    cs_tol = 1e-6 if rtol > 1e-9 else 1e-13
    assert np.max(np.abs(ca - d) / d) <= cs_tol and np.max(np.abs(cb - d) / d) <= cs_tol
    G = Xh.T @ Xh
    assert np.linalg.norm(Ra.T @ Ra - G) / np.trace(G) <= gram_tol
    Ro = otsqr.tsqr_r_final(Xh, leaf_rows=4096)
    assert np.abs(Ra - Ro).max() <= rtol * np.abs(Ro).max()


def test_noalloc_two_calls_second_smaller(lib):
    # 2,000,000 x 128: the default tree would not fit the scratch array, so the
    # slabs are lengthened; then a smaller input on the same array.
    X1 = synth.random_matrix(2_000_000, 128, dtype=torch.float32, seed_tag=301).cuda()
    _check(lib, X1, lib.F32, 2e-5, 1e-6)
    del X1
    X2 = synth.random_matrix(300_001, 25, dtype=torch.float32, seed_tag=302).cuda()
    _check(lib, X2, lib.F32, 2e-5, 1e-6)


def test_noalloc_fp64_and_column_major(lib):
    X = synth.random_matrix(200_000, 40, dtype=torch.float64, seed_tag=303).cuda()
    _check(lib, X, lib.F64, 1e-11, 1e-12)
    Xc = synth.random_matrix(64, 100_003, dtype=torch.float32, seed_tag=304).cuda().t()
    _check(lib, Xc, lib.F32, 2e-5, 1e-6)


def test_noalloc_argument_errors(lib):
    R = torch.empty((4, 4), dtype=torch.float64, device="cuda")
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    assert lib.tsnmf_tsqr_r_noalloc(None, 10, 4, 4, lib.F32, R) == -1
    assert lib.tsnmf_tsqr_r_noalloc(X, 10, 4, 3, lib.F32, R) == -4
    assert lib.tsnmf_tsqr_r_noalloc(X, 10, 4, 4, lib.BF16, R) == -5
    assert lib.tsnmf_tsqr_r_noalloc(X, 10, 300, 300, lib.F32, R) == 4
