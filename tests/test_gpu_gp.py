"""GPU parity of tsnmf_gauss_proj (Sec. 2.3; Sec. 3.2, Algorithm 1) against the
CPU oracle (oracle.philox + oracle.gauss_proj), through the C ABI.

Both sides implement Philox4x32-10 and Box-Muller from their published
definitions; the device uses the hardware log2 / sin / cos / sqrt in FP32, the
oracle libm in FP64, so G agrees to ~1e-6 relative.

Tolerances (normwise, ||Y_gpu - Y_ref||_F / ||Y_ref||_F):
  FP32 vector path: 1e-5.  Per entry the FP32 accumulation over the ~m/2048
    rows of one workgroup contributes ~ u sqrt(rows) ~ 6e-8 * 100, and the G
    difference ~1e-6; the workgroup partials are added in FP64.
  BF16 matrix-core path against the oracle on the same BF16 inputs (G rounded
    to BF16 by the oracle): 5e-4.  Entries of G whose FP32 value lies within
    ~1e-6 of a BF16 rounding boundary may round the other way (probability
    ~2.5e-4 per entry, 2^-8 relative each), giving ~6e-5 normwise.
  BF16 path against the FP64 oracle on FP32 inputs (total error of the BF16
    projection): 1e-2, reported.
"""

import numpy as np
import pytest
import torch

from oracle import gauss_proj as ogp
from oracle import philox as oph
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu


def to_bf16(a):
    """Round to bfloat16 (nearest even) through FP32, returned as FP64."""
    x = np.asarray(a, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def _normwise(A, B):
    return float(np.linalg.norm(A - B) / np.linalg.norm(B))


def _gp(lib, X, k, seed, mode=None, row_offset=0, colsum=False):
    torch.cuda.synchronize()
    Y, cs = lib.gauss_proj(X, k, seed, mode=mode, row_offset=row_offset, with_colsum=colsum)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64), (cs.cpu().numpy() if cs is not None else None)


@pytest.mark.parametrize("m,n,k", [(50_003, 25, 64), (20_000, 1, 8), (33_333, 7, 512), (40_001, 128, 512),
                                   (3, 5, 4), (100, 128, 1028)])
def test_simd_fp32_matches_oracle(lib, m, n, k):
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=31, dist="lognormal")
    Yg, csg = _gp(lib, X.cuda(), k, 14026964, mode=lib.GP_SIMD_F32, colsum=True)
    Yo = ogp.gauss_proj(X.numpy(), k, 14026964)
    assert _normwise(Yg, Yo) <= 1e-5
    d = np.abs(X.numpy().astype(np.float64)).sum(0)
    assert np.max(np.abs(csg - d) / d) <= 1e-12


@pytest.mark.parametrize("m,n,k", [(50_003, 25, 64), (33_333, 128, 512), (1000, 3, 1028)])
def test_mfma_bf16_matches_oracle(lib, m, n, k):
    X32 = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=32, dist="uniform")
    Xb = X32.to(torch.bfloat16)
    Yg, _ = _gp(lib, Xb.cuda(), k, 99, mode=lib.GP_MFMA_BF16)
    Xbh = Xb.float().numpy().astype(np.float64)
    G = oph.gaussian_matrix(99, 0, m, k)
    Yk = to_bf16(G).T @ Xbh                      # same BF16 inputs
    assert _normwise(Yg, Yk) <= 5e-4
    Yt = ogp.gauss_proj(X32.numpy(), k, 99)       # FP64 oracle on the FP32 inputs
    assert _normwise(Yg, Yt) <= 1e-2


def test_mfma_from_fp32_input(lib):
    """FP32 input on the matrix cores: X is rounded to BF16 while staged."""
    X = synth.random_matrix(20_000, 40, dtype=torch.float32, seed_tag=33)
    Yg, _ = _gp(lib, X.cuda(), 128, 5, mode=lib.GP_MFMA_BF16)
    Xb = X.to(torch.bfloat16).float().numpy().astype(np.float64)
    Yk = to_bf16(oph.gaussian_matrix(5, 0, 20_000, 128)).T @ Xb
    assert _normwise(Yg, Yk) <= 5e-4


@pytest.mark.parametrize("mode", ["simd", "mfma"])
def test_row_offset_shards_add_up(lib, mode):
    """G depends on the global row only: projecting two row shards with their
    offsets and adding gives the projection of the whole matrix."""
    md = lib.GP_SIMD_F32 if mode == "simd" else lib.GP_MFMA_BF16
    X = synth.random_matrix(30_000, 16, dtype=torch.float32, seed_tag=34).cuda()
    Y, _ = _gp(lib, X, 64, 7, mode=md)
    Y1, _ = _gp(lib, X[:12_345], 64, 7, mode=md)
    Y2, _ = _gp(lib, X[12_345:], 64, 7, mode=md, row_offset=12_345)
    assert _normwise(Y1 + Y2, Y) <= 1e-5
    Yo = ogp.gauss_proj(X[12_345:].cpu().numpy(), 64, 7, row0=12_345)
    if mode == "simd":
        assert _normwise(Y2, Yo) <= 1e-5


def test_deterministic(lib):
    X = synth.random_matrix(77_777, 32, dtype=torch.float32, seed_tag=35).cuda()
    for md in (lib.GP_SIMD_F32, lib.GP_MFMA_BF16):
        A, _ = _gp(lib, X, 256, 3, mode=md)
        B, _ = _gp(lib, X, 256, 3, mode=md)
        assert np.array_equal(A, B)


def test_invalid_arguments(lib):
    X = torch.zeros((10, 4), dtype=torch.float32, device="cuda")
    Y = torch.empty((4, 8), dtype=torch.float32, device="cuda")
    assert lib.tsnmf_gauss_proj(None, 10, 4, 4, lib.F32, 8, 1, 0, Y) == -1
    assert lib.tsnmf_gauss_proj(X, 10, 4, 4, lib.F64, 8, 1, 0, Y) == -5
    assert lib.tsnmf_gauss_proj(X, 10, 4, 4, lib.BF16 | lib.GP_SIMD_F32, 8, 1, 0, Y) == -5
    assert lib.tsnmf_gauss_proj(X, 10, 4, 4, lib.F32, 6, 1, 0, Y) == -6
    assert lib.tsnmf_gauss_proj(X, 10, 4, 4, lib.F32, 8, 1, -1, Y) == -8
    assert lib.tsnmf_gauss_proj(X, 10, 4, 4, lib.F32, 8, 1, 0, None) == -9


def test_projection_workload_full_size_sampled(lib):
    """The projection workload at full size (20,000,000 x 128, k = 512, BF16 on
    the matrix cores and FP32 on the vector units): rows 4q..4q+3 of Y for two
    column groups q, recomputed by the oracle over all rows."""
    d = synth.projection(device="cuda")
    X = d["X"]
    Xb = X.to(torch.bfloat16)
    seed = 14026964
    Yb, _ = _gp(lib, Xb, 512, seed, mode=lib.GP_MFMA_BF16)
    Ys, _ = _gp(lib, X, 512, seed, mode=lib.GP_SIMD_F32)
    Xh = X.cpu().numpy()
    for q in (0, 77):
        ref = ogp.gauss_proj_group(Xh, q, seed)
        assert _normwise(Ys[4 * q:4 * q + 4], ref) <= 1e-5
        assert _normwise(Yb[4 * q:4 * q + 4], ref) <= 1e-2
