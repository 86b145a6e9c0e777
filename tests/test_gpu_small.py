"""GPU parity of the n x n steps (SPA, XRAY, GP selection, NNLS, residual) and
of the whole pipeline, against the CPU oracle, through the C ABI.

Selections are index sets: the GPU's ordered K must equal the oracle's exactly
when both see the same input matrix.  Both sides work in FP64; a pick is only
ambiguous when the two best scores agree to ~1e-12 relative, which the inputs
below avoid (their margins are checked).  NNLS: H within 1e-8 relative of the
oracle's Lawson-Hanson solution (the minimiser is unique for full-column-rank
M(:, K); both solvers reach it to ~cond * eps).
"""

import numpy as np
import pytest
import torch

from oracle import nnls as onnls
from oracle import residual as ores
from oracle import select as osel
from oracle import tsqr as otsqr
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu


def _separable(p, n, r, seed, noise=0.0, spread=1.0):
    rng = np.random.default_rng([41, seed])
    K = sorted(rng.choice(n, size=r, replace=False).tolist())
    H = spread * rng.uniform(size=(r, n))
    H[:, K] = np.eye(r)
    W = rng.uniform(size=(p, r))
    return W @ H + noise * rng.uniform(size=(p, n)), K


def _cuda(a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _margins(scores):
    return scores


@pytest.mark.parametrize("p,n,r", [(20, 20, 10), (25, 25, 16), (64, 64, 20), (128, 128, 32), (200, 200, 20)])
def test_spa_matches_oracle(lib, p, n, r):
    M, _ = _separable(max(p, 300), n, r, p + n, noise=1e-3, spread=2.0)
    R = otsqr.tsqr_r_final(M, leaf_rows=1000)[:p]
    d = np.abs(M).sum(0)
    K, score, info = lib.select_spa(_cuda(R), r, colscale=_cuda(d))
    Ko, so, io = osel.spa(R, r, colscale=d)
    assert K.cpu().tolist() == Ko and int(info.item()) == io
    assert np.allclose(score.cpu().numpy(), so, rtol=1e-12)


def test_spa_on_x_equals_spa_on_r(lib):
    """Sec. 2.2: the picks on X D^{-1} and on R D^{-1} are the same."""
    X, K = _separable(256, 40, 8, 3)
    R = otsqr.tsqr_r_final(X, leaf_rows=100)
    d = np.abs(X).sum(0)
    Kx, _, _ = lib.select_spa(_cuda(X), 8, colscale=_cuda(d))
    Kr, _, _ = lib.select_spa(_cuda(R), 8, colscale=_cuda(d))
    assert Kx.cpu().tolist() == Kr.cpu().tolist()
    assert sorted(Kr.cpu().tolist()) == K


def test_spa_early_stop(lib):
    M = np.zeros((4, 6))
    M[0, 1] = 2.0
    M[1, 4] = 1.0
    K, score, info = lib.select_spa(_cuda(M), 4)
    assert K.cpu().tolist() == [1, 4, -1, -1] and int(info.item()) == 2


@pytest.mark.parametrize("n,r", [(12, 4), (25, 8), (40, 10)])
def test_xray_matches_oracle(lib, n, r):
    M, _ = _separable(300, n, r - 1, n, noise=1e-2)
    R = otsqr.tsqr_r_final(M, leaf_rows=100)
    K, info = lib.select_xray(_cuda(R), r)
    Ko, io = osel.xray(R, r)
    assert K.cpu().tolist() == Ko and int(info.item()) == io


def test_gp_select_matches_oracle(lib):
    rng = np.random.default_rng(7)
    Y = rng.standard_normal((512, 128)).astype(np.float32)
    d = rng.uniform(0.5, 2.0, size=128)
    K, counts, info = lib.select_gp(_cuda(Y), 32, colscale=_cuda(d))
    Ko, co, io = osel.gp_select(Y.astype(np.float64), 32, colscale=d)
    assert K.cpu().tolist() == Ko and counts.cpu().tolist() == co.tolist() and int(info.item()) == io


def test_gp_select_fewer_distinct_than_r(lib):
    Y = np.array([[1.0, 5.0, -2.0, 5.0]], dtype=np.float32)
    K, counts, info = lib.select_gp(_cuda(Y), 4)
    assert K.cpu().tolist() == [1, 2, -1, -1] and int(info.item()) == 2


@pytest.mark.parametrize("p,n,r", [(20, 20, 10), (64, 64, 20), (128, 128, 32), (100, 100, 40), (200, 200, 64)])
def test_nnls_matches_oracle(lib, p, n, r):
    M, K = _separable(p, n, r, 50 + n, noise=5e-2)
    Kt = torch.tensor(K, dtype=torch.int32, device="cuda")
    H, res, info = lib.nnls(_cuda(M), Kt)
    H = H.cpu().numpy()
    Ho, ro, io = onnls.nnls_matrix(M, K)
    assert np.abs(H - Ho).max() <= 1e-8 * max(1.0, np.abs(Ho).max())
    assert np.allclose(res.cpu().numpy(), ro, rtol=1e-8, atol=1e-20)
    assert info.cpu().tolist() == io.tolist()
    A = M[:, K]
    for i in range(0, n, 7):
        assert onnls.kkt_violation(A, M[:, i], H[:, i]) <= 1e-10
    rel = lib.residual(_cuda(M), Kt, torch.from_numpy(H).cuda())
    assert abs(float(rel.item()) - ores.relative_residual(M, K, Ho)) <= 1e-12


@pytest.mark.parametrize("p,n,r", [(40, 30, 6), (90, 70, 25), (256, 256, 64)])
def test_nnls_binding_constraints(lib, p, n, r):
    """Columns with negative parts along a picked column, so that many entries
    of H sit on the bound and the step-length logic of Lawson-Hanson runs."""
    M, K = _separable(p, n, r, 70 + r, noise=1e-1)
    W = M[:, K]
    M[:, ::3] -= 0.4 * W[:, [0]]
    M[:, 1::4] -= 0.2 * W[:, [r - 1]]
    Kt = torch.tensor(K, dtype=torch.int32, device="cuda")
    H, res, info = lib.nnls(_cuda(M), Kt)
    H = H.cpu().numpy()
    Ho, ro, io = onnls.nnls_matrix(M, K)
    assert (Ho == 0.0).sum() >= n // 3                      # constraints bind
    assert np.abs(H - Ho).max() <= 1e-8 * max(1.0, np.abs(Ho).max())
    assert np.allclose(res.cpu().numpy(), ro, rtol=1e-8, atol=1e-20)
    assert info.cpu().tolist() == io.tolist()
    A = M[:, K]
    for i in range(0, n, 5):
        assert onnls.kkt_violation(A, M[:, i], H[:, i]) <= 1e-10


def test_nnls_reduced_equals_full(lib):
    """Sec. 2.4: NNLS on R gives the H of NNLS on X."""
    X, K = _separable(2000, 30, 6, 9, noise=1e-2)
    R = otsqr.tsqr_r_final(X, leaf_rows=500)
    Kt = torch.tensor(K, dtype=torch.int32, device="cuda")
    Hr, _, _ = lib.nnls(_cuda(R), Kt)
    Hx, _, _ = onnls.nnls_matrix(X, K)
    assert np.abs(Hr.cpu().numpy() - Hx).max() <= 1e-8 * np.abs(Hx).max()


def test_bad_indices_are_rejected_on_device(lib):
    M = np.eye(5)
    Kt = torch.tensor([0, 7], dtype=torch.int32, device="cuda")
    H, res, info = lib.nnls(_cuda(M), Kt)
    assert np.isnan(H.cpu().numpy()).all() and (info.cpu().numpy() == 2).all()
    rel = lib.residual(_cuda(M), Kt, torch.zeros((2, 5), dtype=torch.float64, device="cuda"))
    assert np.isnan(rel.item())


def test_invalid_arguments(lib):
    M = torch.zeros((4, 4), dtype=torch.float64, device="cuda")
    K = torch.zeros(2, dtype=torch.int32, device="cuda")
    info = torch.zeros(1, dtype=torch.int32, device="cuda")
    assert lib.tsnmf_select_spa(None, 4, 4, 4, None, 2, K, None, info) == -1
    assert lib.tsnmf_select_spa(M, 4, 300, 4, None, 2, K, None, info) == -3
    assert lib.tsnmf_select_spa(M, 4, 4, 3, None, 2, K, None, info) == -4
    assert lib.tsnmf_select_spa(M, 4, 4, 4, None, 5, K, None, info) == -6
    assert lib.tsnmf_select_xray(M, 4, 4, 4, 0, K, info) == -5
    assert lib.tsnmf_nnls(M, 4, 4, 4, K, 2, None, 2) == -7
    assert lib.tsnmf_nnls(M, 4, 4, 4, K, 2, M, 1) == -8


# ---- whole pipeline on the GPU ---------------------------------------------------

def test_pipeline_plain_fp64(lib):
    """100,000 x 20 FP64, r = 10: TSQR (1,000-row leaves, binary tree), SPA on
    R D^{-1}, NNLS, residual -- all on the GPU, against the oracle."""
    d = synth.plain_fp64()
    X = d["X"]
    cfg = lib.TsqrConfig(leaf_rows=1000, tree_arity=2, rows_per_lane=0)
    R, cs = lib.tsqr_r(X.cuda(), config=cfg)
    K, _, info = lib.select_spa(R, 10, colscale=cs)
    H, _, _ = lib.nnls(R, K)
    rel = lib.residual(R, K, H)
    Xh = X.numpy()
    Ro = otsqr.tsqr_r_final(Xh, leaf_rows=1000)
    do = np.abs(Xh).sum(0)
    Ko, so, _ = osel.spa(Ro, 10, colscale=do)
    assert K.cpu().tolist() == Ko                          # bit-identical K
    assert sorted(Ko) == d["K"]                            # the planted columns
    Ho, _, _ = onnls.nnls_matrix(Ro, Ko)
    assert np.abs(H.cpu().numpy() - Ho).max() <= 1e-8 * np.abs(Ho).max()
    assert abs(rel.item() - ores.relative_residual(Ro, Ko, Ho)) <= 1e-10


def test_pipeline_flow_cytometry_fp32(lib):
    """1e6 x 25 FP32 flow-cytometry-shaped data (r = 16): FP32 leaves, FP64 tree,
    SPA, NNLS on the GPU; K equal to the oracle's (on the oracle's R) and the
    planted set."""
    d = synth.flow_cytometry(m=1_000_000)
    X = d["X"]
    R, cs = lib.tsqr_r(X.cuda())
    K, score, _ = lib.select_spa(R, 16, colscale=cs)
    Xh = X.numpy().astype(np.float64)
    Ro = otsqr.tsqr_r_final(Xh, leaf_rows=4096)
    do = np.abs(Xh).sum(0)
    Ko, so, _ = osel.spa(Ro, 16, colscale=do)
    s = np.asarray(so)
    assert np.min(np.abs(np.diff(s)) / s[:-1]) > 1e-6     # picks are not near-ties
    assert K.cpu().tolist() == Ko
    assert sorted(Ko) == d["K"]
    H, _, _ = lib.nnls(R, K)
    Ho, _, _ = onnls.nnls_matrix(Ro, Ko)
    assert np.abs(H.cpu().numpy() - Ho).max() <= 1e-4 * np.abs(Ho).max()


@pytest.mark.parametrize("noisy", [False, True])
def test_paper_example_end_to_end_on_gpu(lib, noisy):
    """The Sec. 4 example at m = 20,000 (n = 200, r = 20; exactly separable, and
    with U[0, 1e-3] noise), the whole path on the GPU: TSQR with column sums
    (FP64, 200 columns), SPA on R D^{-1}, NNLS and the residual.  Against the
    oracle on the same bytes: the same K, equal to the swap rule's
    {0, 1, 20, 30, ..., 190}; the residual vanishes at r = 20 on exact data and
    is at the noise level otherwise; the first 21 greedy XRAY picks contain K."""
    d = synth.paper_example(20_000, noisy=noisy)
    X = d["X"]
    R, cs = lib.tsqr_r(X.cuda())
    K, _, info = lib.select_spa(R, 20, colscale=cs)
    H, _, _ = lib.nnls(R, K)
    rel = lib.residual(R, K, H)
    torch.cuda.synchronize()
    Xh = X.numpy()
    Ro = otsqr.tsqr_r_final(Xh, leaf_rows=1000)
    do = np.abs(Xh).sum(0)
    Ko, _, _ = osel.spa(Ro, 20, colscale=do)
    assert int(info.item()) == 20
    assert K.cpu().tolist() == Ko
    assert sorted(Ko) == d["K"] == [0, 1] + list(range(20, 200, 10))
    Xg = Xh.T @ Xh
    Rg = R.cpu().numpy()
    assert np.linalg.norm(Rg.T @ Rg - Xg) / np.trace(Xg) <= 1e-12
    if noisy:
        Ho, _, _ = onnls.nnls_matrix(Ro, Ko)
        ro = ores.relative_residual(Ro, Ko, Ho)
        assert 0.0 < rel.item() <= 1e-6 and abs(rel.item() - ro) <= 1e-3 * ro
    else:
        assert rel.item() < 1e-20
    Kx, _ = lib.select_xray(R, 21)
    assert set(d["K"]) <= set(Kx.cpu().tolist())
