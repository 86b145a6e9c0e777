"""GPU parity of tsnmf_tsqr_r_batched (many independent TSQRs in one persistent
launch) against the CPU oracle, through the C ABI.

Each matrix of a batch is checked like a single tsnmf_tsqr_r call: R upper
triangular with diag(R) >= 0, ||R^T R - X^T X||_F / ||X||_F^2 <= 1e-6 (FP32 row
blocks, FP64 trees), column 2-norms of R within 1e-5 of those of X, R element-wise
within 2e-5 (relative to max |R|) of the oracle's on well-conditioned inputs, and
l1 column sums within 1e-6.  The batch exercises every width class (16 and 32
with ld = n on the one-wave kernel, other widths up to 64 and up to 128 on the
four-wave kernel), one-slab matrices, m < n, ragged tails, multi-level trees and
strided rows.
"""

import numpy as np
import pytest
import torch

from oracle import tsqr as otsqr
from paper_1402_6964_amd import synth

pytestmark = pytest.mark.gpu


def _check(Rg, csg, Xh, gram_tol=1e-6, elem_tol=2e-5, cs_tol=1e-6, norm_tol=1e-5, name=""):
    X64 = np.asarray(Xh, dtype=np.float64)
    n = X64.shape[1]
    assert Rg.shape == (n, n)
    assert np.all(np.tril(Rg, -1) == 0.0), f"{name}: strict lower triangle must be zero"
    assert np.all(np.diag(Rg) >= 0.0), f"{name}: diag(R) >= 0"
    G = X64.T @ X64
    g = np.linalg.norm(Rg.T @ Rg - G) / np.linalg.norm(X64) ** 2
    assert g <= gram_tol, f"{name}: gram error {g:.3e}"
    cn = np.linalg.norm(X64, axis=0)
    nz = cn > 0
    rel = np.abs(np.linalg.norm(Rg, axis=0)[nz] - cn[nz]) / cn[nz]
    assert rel.max(initial=0.0) <= norm_tol, f"{name}: column-norm error {rel.max():.3e}"
    if elem_tol is not None:
        Ro = otsqr.tsqr_r_final(X64, leaf_rows=4096)
        err = np.abs(Rg - Ro).max() / np.abs(Ro).max()
        assert err <= elem_tol, f"{name}: R element error {err:.3e}"
    if csg is not None:
        d = np.abs(X64).sum(axis=0)
        nzd = d > 0
        rc = np.abs(csg[nzd] - d[nzd]) / d[nzd]
        assert rc.max(initial=0.0) <= cs_tol, f"{name}: colsum error {rc.max():.3e}"


# (m, n, extra columns of the row stride)
MIXED = [
    (100_003, 16, 0), (4_096, 16, 0), (700_001, 16, 0), (5, 16, 0),
    (100_001, 32, 0), (4_095, 32, 0), (300_007, 32, 0),
    (90_001, 64, 0), (8_192, 64, 0), (8_193, 64, 0), (20_000, 48, 0), (33, 33, 0),
    (50_001, 128, 0), (16_384, 128, 0), (140_000, 128, 0), (100, 128, 0), (20_011, 100, 0),
    (60_000, 16, 3), (40_000, 32, 5), (30_001, 7, 0), (3, 1, 0), (10_000, 2, 0), (12_345, 65, 0),
]


def _mixed(seed_tag=40):
    mats = []
    for q, (m, n, extra) in enumerate(MIXED):
        full = synth.random_matrix(m, n + extra, dtype=torch.float32, seed_tag=seed_tag + q, dist="uniform")
        mats.append(full)
    return mats


def _device_views(mats):
    out = []
    for (m, n, extra), full in zip(MIXED, mats):
        d = full.cuda()
        out.append(d[:, :n] if extra else d)
    return out


def test_mixed_batch_matches_oracle(lib):
    mats = _mixed()
    dv = _device_views(mats)
    b = lib.Batch(dv)
    torch.cuda.synchronize()
    b.run()
    torch.cuda.synchronize()
    for (m, n, extra), full, (R, cs) in zip(MIXED, mats, b.results()):
        X = full[:, :n].numpy()
        # m < n: R^T R = X^T X still holds; R is not unique there, so no element check
        _check(R.cpu().numpy(), cs.cpu().numpy(), X, elem_tol=None if m < n else 2e-5, name=f"{m}x{n}")


@pytest.mark.parametrize("shifts", [(1, 2, 1, 2), (3, 3, 3, 3), (8, 0, 8, 0)])
def test_slab_shifts_match_oracle(lib, shifts):
    """tsnmf_tsqr_r_batched_ex with longer slabs per width class (fewer
    leaves and tree levels, down to one slab per matrix at shift 8): the same
    bars as the default geometry."""
    mats = _mixed(seed_tag=60)
    dv = _device_views(mats)
    b = lib.Batch(dv)
    b.run(config=lib.batch_config(shifts))
    torch.cuda.synchronize()
    for (m, n, extra), full, (R, cs) in zip(MIXED, mats, b.results()):
        X = full[:, :n].numpy()
        _check(R.cpu().numpy(), cs.cpu().numpy(), X, elem_tol=None if m < n else 2e-5, name=f"{shifts} {m}x{n}")


def test_batch_equals_single_calls(lib):
    """The same matrices through tsnmf_tsqr_r one by one: R agrees to FP32
    rounding (the slab heights and tree shapes differ)."""
    mats = _mixed(seed_tag=80)
    dv = _device_views(mats)
    res = lib.tsqr_r_batched(dv)
    torch.cuda.synchronize()
    for (m, n, extra), X, (Rb, csb) in zip(MIXED, dv, res):
        if m < n:
            continue
        Rs, css = lib.tsqr_r(X)
        Rb, Rs = Rb.cpu().numpy(), Rs.cpu().numpy()
        assert np.abs(Rb - Rs).max() <= 4e-5 * np.abs(Rs).max(), f"{m}x{n}"
        assert np.allclose(csb.cpu().numpy(), css.cpu().numpy(), rtol=2e-6, atol=0)


def test_repeat_is_deterministic(lib):
    mats = _device_views(_mixed(seed_tag=120))
    b = lib.Batch(mats)
    b.run()
    first = [(R.cpu().numpy().copy(), c.cpu().numpy().copy()) for R, c in b.results()]
    for _ in range(2):
        b.run()
        for (R0, c0), (R, c) in zip(first, b.results()):
            assert np.array_equal(R0, R.cpu().numpy()) and np.array_equal(c0, c.cpu().numpy())


def test_graph_capture_and_replay(lib):
    """Captured once, replayed with new data and new shapes written into the
    same device arrays; every replay is checked against an eager call."""
    shapes = [(200_000, 16), (120_001, 32), (80_000, 64), (60_000, 128), (30_000, 40), (9_000, 100)]
    mats = [synth.random_matrix(m, n, dtype=torch.float32, seed_tag=160 + q, dist="uniform").cuda()
            for q, (m, n) in enumerate(shapes)]
    lib.reserve_batched(len(mats), sum(m for m, _ in shapes))
    b = lib.Batch(mats)
    eager = lib.Batch(mats)
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        b.run()                        # warm-up outside capture (kernel attributes)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    for rep in range(4):
        if rep == 1:
            for X in mats:
                X.mul_(2.0)            # new data
        if rep == 2:                   # new shapes: fewer rows, read on the device
            b.m.copy_(torch.tensor([m // 3 + 1 for m, _ in shapes], dtype=torch.int64))
            eager.m.copy_(b.m)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        eager.run()
        torch.cuda.synchronize()
        rows = [int(v) for v in b.m.cpu()]
        for q, ((R, cs), (Re, cse)) in enumerate(zip(b.results(), eager.results())):
            Rn = R.cpu().numpy()
            assert np.array_equal(Rn, Re.cpu().numpy()), f"replay {rep} matrix {q}"
            assert np.array_equal(cs.cpu().numpy(), cse.cpu().numpy())
            if q in (0, 3):
                _check(Rn, cs.cpu().numpy(), mats[q][:rows[q]].cpu().numpy(), name=f"replay {rep} matrix {q}")


def test_invalid_entries_give_nan(lib):
    good = synth.random_matrix(10_000, 16, dtype=torch.float32, seed_tag=200).cuda()
    other = synth.random_matrix(5_000, 8, dtype=torch.float32, seed_tag=201).cuda()
    b = lib.Batch([good, other, good])
    b.n.copy_(torch.tensor([16, 8, 16], dtype=torch.int64))
    b.ld.copy_(torch.tensor([16, 4, 16], dtype=torch.int64))    # matrix 1: ld < n
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    assert np.isnan(res[1][0].cpu().numpy()).all() and np.isnan(res[1][1].cpu().numpy()).all()
    for q in (0, 2):
        _check(res[q][0].cpu().numpy(), res[q][1].cpu().numpy(), good.cpu().numpy(), name=str(q))


def test_huge_row_stride_every_wide_class(lib):
    """Row stride 2^23 (rows 32 MiB apart) for a 64- and a 128-column matrix
    in the same store: both wide classes load each 64-row chunk with 64-bit
    addresses and regroup it through LDS, so any stride is served."""
    ld = 1 << 23
    m = 100
    store = torch.zeros((m, ld), dtype=torch.float32, device="cuda")
    A = synth.random_matrix(m, 128, dtype=torch.float32, seed_tag=202)
    store[:, :128] = A.cuda()
    wide = synth.random_matrix(1_000, 128, dtype=torch.float32, seed_tag=203).cuda()
    b = lib.Batch([store[:, :64], store[:, :128], wide])
    assert b.ld.cpu().tolist() == [ld, ld, 128]
    b.run()
    torch.cuda.synchronize()
    res = b.results()
    _check(res[0][0].cpu().numpy(), res[0][1].cpu().numpy(), A[:, :64].numpy(), name="n = 64, ld = 2^23")
    _check(res[1][0].cpu().numpy(), res[1][1].cpu().numpy(), A.numpy(), name="n = 128, ld = 2^23")
    _check(res[2][0].cpu().numpy(), res[2][1].cpu().numpy(), wide.cpu().numpy(), name="n = 128, ld = 128")
    del store


def test_without_colsums(lib):
    X = synth.random_matrix(50_000, 32, dtype=torch.float32, seed_tag=210).cuda()
    (R, cs), = lib.tsqr_r_batched([X], with_colsum=False)
    assert cs is None
    _check(R.cpu().numpy(), None, X.cpu().numpy())


def test_argument_errors(lib):
    a = torch.zeros(2, dtype=torch.int64, device="cuda")
    assert lib.tsnmf_tsqr_r_batched(0, a, a, a, a, lib.F32, a) == -1
    assert lib.tsnmf_tsqr_r_batched(lib.MAX_BATCH + 1, a, a, a, a, lib.F32, a) == -1
    assert lib.tsnmf_tsqr_r_batched(2, None, a, a, a, lib.F32, a) == -2
    assert lib.tsnmf_tsqr_r_batched(2, a, None, a, a, lib.F32, a) == -3
    assert lib.tsnmf_tsqr_r_batched(2, a, a, None, a, lib.F32, a) == -4
    assert lib.tsnmf_tsqr_r_batched(2, a, a, a, None, lib.F32, a) == -5
    assert lib.tsnmf_tsqr_r_batched(2, a, a, a, a, lib.F64, a) == -6
    assert lib.tsnmf_tsqr_r_batched(2, a, a, a, a, lib.F32 | lib.COL_MAJOR, a) == -6
    assert lib.tsnmf_tsqr_r_batched(2, a, a, a, a, lib.F32, None) == -7
    for bad in ((9, 0, 0, 0), (0, -1, 0, 0)):
        assert lib.tsnmf_tsqr_r_batched_ex(2, a, a, a, a, lib.F32, a, None, lib.batch_config(bad)) == -8
    cfg = lib.batch_config((0, 0, 0, 0))
    cfg.reserved[2] = 1
    assert lib.tsnmf_tsqr_r_batched_ex(2, a, a, a, a, lib.F32, a, None, cfg) == -8
    assert lib.tsnmf_tsqr_r_batched_ex(2, a, a, a, a, lib.F32, None, None, cfg) == -7
    assert lib.tsnmf_reserve_batched(0, 10) == -1
    assert lib.tsnmf_reserve_batched(4, -1) == -2


def test_batched_workload_full_size(lib):
    """The full batched workload (512 matrices, m log-uniform in [1e4, 2e6],
    n in {16, 32, 64, 128}, 44.5 GB) in one graph-captured call, as bench.py
    times it.  Every matrix: column 2-norms of R and l1 column sums against
    FP64 sums of X on the device; R upper triangular with diag >= 0.  The
    shortest matrix of each width: R against the oracle."""
    shapes = synth.batch_shapes()
    mats = [synth.batch_matrix(q, m, n, device="cuda")["X"] for q, (m, n) in enumerate(shapes)]
    b = lib.Batch(mats)
    b.run()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        b.run()
    g.replay()
    torch.cuda.synchronize()
    res = b.results()
    worst_norm, worst_cs = 0.0, 0.0
    for X, (R, cs) in zip(mats, res):
        Rn = R.cpu().numpy()
        assert np.all(np.tril(Rn, -1) == 0.0) and np.all(np.diag(Rn) >= 0.0)
        X64 = X.double()
        cn = torch.sqrt((X64 * X64).sum(0)).cpu().numpy()
        d = X64.abs().sum(0).cpu().numpy()
        worst_norm = max(worst_norm, float(np.max(np.abs(np.linalg.norm(Rn, axis=0) - cn) / cn)))
        worst_cs = max(worst_cs, float(np.max(np.abs(cs.cpu().numpy() - d) / d)))
        del X64
    assert worst_norm <= 1e-5, worst_norm
    assert worst_cs <= 1e-6, worst_cs
    for n in (16, 32, 64, 128):
        q = min((i for i, s in enumerate(shapes) if s[1] == n), key=lambda i: shapes[i][0])
        Xh = mats[q].cpu().numpy()
        _check(res[q][0].cpu().numpy(), res[q][1].cpu().numpy(), Xh, name=f"{shapes[q]}")
