"""GPU parity of tsnmf_gauss_proj (Sec. 2.3; Sec. 3.2, Algorithm 1) against the
CPU oracle (oracle.philox + oracle.gauss_proj), through the C ABI, entry by
entry.

Both sides implement Philox4x32-10 and Box-Muller from their published
definitions.  The device forms G in FP32 with the hardware log2, sqrt, sin and
cos; the oracle in FP64 with libm.  The uniforms are exact on both sides, so G
differs only by the error of those functions: |G_gpu - G| <= EPS_G * rho,
rho = sqrt(-2 ln u) the Box-Muller radius of the entry's pair (recovered from
the oracle's G as hypot of the pair).  The identity tests below measure G
itself: projecting an identity block makes every Y entry one G entry, exactly.

Per-entry bound of Y = G^T X (l, j), FP32 vector path:
    |Y_gpu - Y| <= EPS_G (rho^T |X|) + C_ACC u sqrt(L) (|G|^T |X|) + u |Y|
  with u = 2^-24, L the rows one FP32 accumulator sums (a workgroup takes
  ceil(m / 2048) rows, rounded up to 64), the workgroup partials added in
  FP64, and C_ACC = 8 on the probabilistic rounding-error bound of a sum of L
  terms (Higham & Mary, SIAM J. Sci. Comput. 2019).
BF16 matrix-core path, against the oracle on the same BF16-rounded inputs
(G rounded by the oracle from its FP64 value, X rounded to nearest even):
    |Y_gpu - Y_k| <= sum over entries of G within EPS_G rho of a BF16 rounding
                     boundary of ulp_bf16(G) |X|  +  the two accumulation terms,
  since those entries may round the other way on the device.  Against the
  FP64 oracle on the FP32 inputs (the total error of the BF16 projection) the
  normwise error is reported and held to 1e-2.
"""

import numpy as np
import pytest
import torch

from oracle import gauss_proj as ogp
from oracle import philox as oph
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
EPS_G = 2.0 ** -18       # hardware log2 / sqrt / sin / cos, relative to the radius
C_ACC = 8.0


def to_bf16(a):
    """Round to bfloat16 (nearest even) through FP32, returned as FP64."""
    x = np.asarray(a, dtype=np.float32)
    b = x.view(np.uint32).astype(np.uint64)
    b = ((b + 0x7FFF + ((b >> 16) & 1)) >> 16) << 16
    return b.astype(np.uint32).view(np.float32).astype(np.float64)


def bf16_ulp(a):
    """Spacing of bfloat16 numbers at |a| (8 significant bits)."""
    a = np.abs(np.asarray(a, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(a, 2.0 ** -126)))
    return 2.0 ** (e - 7)


def radius(G):
    """Box-Muller radius of every entry: columns (4q, 4q+1) and (4q+2, 4q+3)
    share one, and cos^2 + sin^2 = 1 recovers it from the pair."""
    P = G.reshape(G.shape[0], -1, 2)
    return np.repeat(np.hypot(P[..., 0], P[..., 1]), 2, axis=1)


def near_bf16_boundary(G):
    """Entries whose FP64 value lies within EPS_G rho of a BF16 rounding
    boundary (a midpoint between neighbouring BF16 numbers): the device's FP32
    G may round to the other neighbour there."""
    g = np.asarray(G, dtype=np.float64)
    lo = to_bf16(g)
    ulp = bf16_ulp(lo)
    mid_up, mid_dn = lo + ulp / 2, lo - bf16_ulp(lo - ulp / 2) / 2
    d = np.minimum(np.abs(g - mid_up), np.abs(g - mid_dn))
    return d <= EPS_G * radius(g) + 2.0 ** -30 * np.abs(g)


def acc_rows(m):
    """Rows summed by one FP32 accumulator (upper bound of the launch's)."""
    return max(64, -(-m // 2048) + 64)


def _gp(lib, X, k, seed, mode=None, row_offset=0, colsum=False):
    torch.cuda.synchronize()
    Y, cs = lib.gauss_proj(X, k, seed, mode=mode, row_offset=row_offset, with_colsum=colsum)
    torch.cuda.synchronize()
    return Y.cpu().numpy().astype(np.float64), (cs.cpu().numpy() if cs is not None else None)


class Sums:
    """Oracle projection and the quantities of the per-entry bounds, summed
    over row chunks: Y = G^T X (FP64), Yk = bf16(G)^T bf16(X), |G|^T |X|,
    rho^T |X|, |bf16 G|^T |bf16 X| and the BF16 boundary term."""

    def __init__(self, X, seed, cols=None, row0=0, chunk=1 << 17, Xb=None):
        X = np.asarray(X)
        m, n = X.shape
        groups = cols
        kk = 4 * len(groups)
        self.Y = np.zeros((kk, n))
        self.Yk = np.zeros((kk, n))
        self.A = np.zeros((kk, n))
        self.P = np.zeros((kk, n))
        self.Ab = np.zeros((kk, n))
        self.B = np.zeros((kk, n))
        for i in range(0, m, chunk):
            C = np.asarray(X[i:i + chunk], dtype=np.float64)
            rows = np.arange(row0 + i, row0 + i + C.shape[0], dtype=np.uint64)
            G = np.concatenate([oph.gaussian_block(seed, rows, q) for q in groups], axis=1)
            Gb = to_bf16(G)
            Cb = to_bf16(C) if Xb is None else np.asarray(Xb[i:i + chunk], dtype=np.float64)
            aC, aCb = np.abs(C), np.abs(Cb)
            self.Y += G.T @ C
            self.Yk += Gb.T @ Cb
            self.A += np.abs(G).T @ aC
            self.P += radius(G).T @ aC
            self.Ab += np.abs(Gb).T @ aCb
            self.B += (near_bf16_boundary(G) * bf16_ulp(G)).T @ aCb
        self.L = acc_rows(m)

    def bound_f32(self):
        return EPS_G * self.P + C_ACC * U32 * np.sqrt(self.L) * self.A + U32 * np.abs(self.Y) + 1e-30

    def bound_bf16(self):
        return self.B + C_ACC * U32 * np.sqrt(self.L) * self.Ab + U32 * np.abs(self.Yk) + 1e-30


def all_groups(k):
    return list(range(k // 4))


# ---- G itself -------------------------------------------------------------------

@pytest.mark.parametrize("k", [512, 128, 32])
@pytest.mark.parametrize("offset", [0, 123_457, 2 ** 32 - 64, 3 * 2 ** 40 + 11])
def test_gaussian_entries_simd(lib, offset, k):
    """Y of a 128 x 128 identity block at row offset o is G(o + j, l) exactly
    (one nonzero product per sum): every entry of G within EPS_G rho of the
    oracle's, including rows whose index crosses 2^32 (the high counter word).
    k = 128 and 32 run the layout in which lanes split the rows."""
    X = torch.eye(128, dtype=torch.float32, device="cuda")
    Y, _ = _gp(lib, X, k, 0x1234_5678_9ABC_DEF0, mode=lib.GP_SIMD_F32, row_offset=offset)
    G = oph.gaussian_matrix(0x1234_5678_9ABC_DEF0, offset, 128, k)       # rows o .. o + 127
    err = np.abs(Y.T - G) / radius(G)
    print(f"max |G_gpu - G| / rho = {err.max():.3e}")
    assert err.max() <= EPS_G


@pytest.mark.parametrize("k", [512, 256, 128, 64])
@pytest.mark.parametrize("offset", [0, 2 ** 32 - 64])
def test_gaussian_entries_bf16(lib, offset, k):
    """On the matrix cores the identity block gives bf16(G_gpu) exactly: equal
    to the BF16 rounding of the oracle's G except at entries within EPS_G rho
    of a rounding boundary, which may differ by one BF16 step.  k = 64 and
    128 run the mode in which 8 or 4 waves share a slice of G through LDS."""
    X = torch.eye(128, dtype=torch.bfloat16, device="cuda")
    Y, _ = _gp(lib, X, k, 99, mode=lib.GP_MFMA_BF16, row_offset=offset)
    G = oph.gaussian_matrix(99, offset, 128, k)
    Gb = to_bf16(G)
    amb = near_bf16_boundary(G)
    d = np.abs(Y.T - Gb)
    assert np.all(d[~amb] == 0.0)
    assert np.all(d[amb] <= bf16_ulp(G)[amb] * 1.0000001)
    assert amb.mean() < 2e-2


# ---- Y, entry by entry -------------------------------------------------------------

@pytest.mark.parametrize("m,n,k", [(50_003, 25, 64), (20_000, 1, 8), (33_333, 7, 512), (40_001, 128, 512),
                                   (3, 5, 4), (100, 128, 1028), (30_001, 200, 64), (10_000, 256, 516),
                                   (7_777, 128, 32), (12_001, 40, 100), (6_001, 30, 200), (4_000, 50, 300)])
def test_simd_fp32_matches_oracle(lib, m, n, k):
    X = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=31, dist="lognormal")
    Yg, csg = _gp(lib, X.cuda(), k, 14026964, mode=lib.GP_SIMD_F32, colsum=True)
    s = Sums(X.numpy(), 14026964, cols=all_groups(k))
    ratio = np.abs(Yg - s.Y) / s.bound_f32()
    print(f"max error / bound = {ratio.max():.3f}; normwise {np.linalg.norm(Yg - s.Y) / np.linalg.norm(s.Y):.2e}")
    assert ratio.max() <= 1.0
    assert np.linalg.norm(Yg - s.Y) / np.linalg.norm(s.Y) <= 1e-5
    d = np.abs(X.numpy().astype(np.float64)).sum(0)
    assert np.max(np.abs(csg - d) / d) <= 1e-12


@pytest.mark.parametrize("m,n,k", [(50_003, 25, 64), (33_333, 128, 512), (1000, 3, 1028), (20_000, 256, 128),
                                   (5_000, 130, 64), (7_001, 40, 4), (12_345, 128, 36), (6_000, 33, 100),
                                   (9_001, 70, 200), (3, 5, 4), (65, 7, 100)])
def test_mfma_bf16_matches_oracle(lib, m, n, k):
    X32 = synth.random_matrix(m, n, dtype=torch.float32, seed_tag=32, dist="uniform")
    Xb = X32.to(torch.bfloat16)
    Yg, _ = _gp(lib, Xb.cuda(), k, 99, mode=lib.GP_MFMA_BF16)
    s = Sums(Xb.float().numpy(), 99, cols=all_groups(k))
    ratio = np.abs(Yg - s.Yk) / s.bound_bf16()
    print(f"max error / bound = {ratio.max():.3f}")
    assert ratio.max() <= 1.0
    Yt = ogp.gauss_proj(X32.numpy(), k, 99)       # FP64 oracle on the FP32 inputs
    assert np.linalg.norm(Yg - Yt) / np.linalg.norm(Yt) <= 1e-2


@pytest.mark.parametrize("width,c0,n", [(131, 1, 128), (130, 2, 64), (130, 1, 64), (64, 0, 63)])
def test_mfma_bf16_strided_views(lib, width, c0, n):
    """BF16 column slices of a wider matrix: row length `width` (odd or even)
    and a first column c0 that leaves the rows 2-byte aligned only (c0 odd) or
    4-byte aligned (c0 even), so both the paired dword loads and the
    element-wise loads run; the column sums of the same call are the FP64 sums
    of the BF16 values."""
    m, k = 9_001, 128
    W = synth.random_matrix(m, width, dtype=torch.float32, seed_tag=36, dist="lognormal").to(torch.bfloat16)
    Wd = W.cuda()
    X = Wd[:, c0:c0 + n]
    assert X.stride(0) == width and (X.data_ptr() % 4 == 0) == (c0 % 2 == 0)
    Yg, csg = _gp(lib, X, k, 123, mode=lib.GP_MFMA_BF16, colsum=True)
    Xh = W[:, c0:c0 + n].float().numpy()
    s = Sums(Xh, 123, cols=all_groups(k))
    assert (np.abs(Yg - s.Yk) / s.bound_bf16()).max() <= 1.0
    d = np.abs(Xh.astype(np.float64)).sum(0)
    assert np.max(np.abs(csg - d) / d) <= 1e-12


def test_mfma_from_fp32_input(lib):
    """FP32 input on the matrix cores: X is rounded to BF16 (nearest even) while
    staged, so the reference is the oracle on bf16(X)."""
    X = synth.random_matrix(20_000, 40, dtype=torch.float32, seed_tag=33)
    Yg, _ = _gp(lib, X.cuda(), 128, 5, mode=lib.GP_MFMA_BF16)
    s = Sums(X.numpy(), 5, cols=all_groups(128))       # Sums rounds X to BF16 for Yk
    assert (np.abs(Yg - s.Yk) / s.bound_bf16()).max() <= 1.0


@pytest.mark.parametrize("mode", ["simd", "mfma"])
def test_row_offset_shards_add_up(lib, mode):
    """G depends on the global row only: projecting two row shards with their
    offsets and adding gives the projection of the whole matrix."""
    md = lib.GP_SIMD_F32 if mode == "simd" else lib.GP_MFMA_BF16
    X = synth.random_matrix(30_000, 16, dtype=torch.float32, seed_tag=34).cuda()
    Y, _ = _gp(lib, X, 64, 7, mode=md)
    Y1, _ = _gp(lib, X[:12_345], 64, 7, mode=md)
    Y2, _ = _gp(lib, X[12_345:], 64, 7, mode=md, row_offset=12_345)
    assert np.linalg.norm(Y1 + Y2 - Y) / np.linalg.norm(Y) <= 1e-5
    s = Sums(X[12_345:].cpu().numpy(), 7, cols=all_groups(64), row0=12_345)
    if mode == "simd":
        assert (np.abs(Y2 - s.Y) / s.bound_f32()).max() <= 1.0
    else:
        assert (np.abs(Y2 - s.Yk) / s.bound_bf16()).max() <= 1.0


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


# Column groups q of the full-size check: rows 4q .. 4q + 3 of Y, every column.
FULL_GROUPS = [0, 1, 37, 77, 101, 127]


@pytest.mark.timeout(400)
def test_projection_workload_full_size_sampled(lib):
    """The projection workload at full size (20,000,000 x 128, k = 512, BF16 on
    the matrix cores and FP32 on the vector units, the launch bench.py times):
    24 of the 512 rows of Y (six Philox column groups spread over the range),
    every one of the 128 columns, recomputed by the oracle over all rows and
    compared entry by entry with the bounds above (and normwise)."""
    d = synth.projection(device="cuda")
    X = d["X"]
    Xb = X.to(torch.bfloat16)
    seed = 14026964
    Yb, _ = _gp(lib, Xb, 512, seed, mode=lib.GP_MFMA_BF16)
    Ys, _ = _gp(lib, X, 512, seed, mode=lib.GP_SIMD_F32)
    Xbh = Xb.float().cpu().numpy()                # the BF16 rounding of X, as FP32 values
    del Xb
    s = Sums(X.cpu().numpy(), seed, cols=FULL_GROUPS, chunk=1 << 19, Xb=Xbh)
    rows = np.concatenate([np.arange(4 * q, 4 * q + 4) for q in FULL_GROUPS])
    rs = np.abs(Ys[rows] - s.Y) / s.bound_f32()
    rb = np.abs(Yb[rows] - s.Yk) / s.bound_bf16()
    print(f"FP32: max error / bound {rs.max():.3f}; BF16: {rb.max():.3f}")
    assert rs.max() <= 1.0 and rb.max() <= 1.0
    assert np.linalg.norm(Ys[rows] - s.Y) / np.linalg.norm(s.Y) <= 1e-5
    assert np.linalg.norm(Yb[rows] - s.Yk) / np.linalg.norm(s.Yk) <= 5e-4
    assert np.linalg.norm(Yb[rows] - s.Y) / np.linalg.norm(s.Y) <= 1e-2


@pytest.mark.parametrize("m,k,off", [(100_003, 512, 0), (5, 4, 2 ** 32 - 2), (1_000_000, 64, 777)])
def test_generator_colsum(lib, m, k, off):
    """tsnmf_gauss_colsum (G^T 1, the generator alone): against the oracle's
    column sums of G, entry by entry with the bound of a projection of a column
    of ones, and against tsnmf_gauss_proj of that column on the vector units."""
    s = lib.gauss_colsum(m, k, 21, row_offset=off)
    torch.cuda.synchronize()
    s = s.cpu().numpy().astype(np.float64)
    ones = np.ones((m, 1), dtype=np.float32)
    ref = Sums(ones, 21, cols=all_groups(k), row0=off)
    assert (np.abs(s - ref.Y[:, 0]) / ref.bound_f32()[:, 0]).max() <= 1.0
    Yp, _ = _gp(lib, torch.ones((m, 1), dtype=torch.float32, device="cuda"), k, 21, mode=lib.GP_SIMD_F32,
                row_offset=off)
    assert (np.abs(s - Yp[:, 0]) / ref.bound_f32()[:, 0]).max() <= 2.0
    assert lib.tsnmf_gauss_colsum(0, k, 21, 0, torch.empty(k, device="cuda")) == -1
    assert lib.tsnmf_gauss_colsum(m, 6, 21, 0, torch.empty(k, device="cuda")) == -2
