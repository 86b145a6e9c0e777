"""Seeded synthetic inputs shaped like the paper's workloads.

This module only draws random numbers and assembles X = W H + N; it contains
none of the method's arithmetic (no QR, projection, selection or NNLS), so the
HIP path and the CPU oracle can both consume what it produces.

Small parameters (the planted index set K, the coefficient matrix H, bump
centres and widths) come from numpy generators keyed by
SeedSequence([14026964, tag, ...]); the tall factors W and the noise N are drawn
with a torch generator seeded the same way, on the device the caller names, in
row chunks, so multi-GB inputs can be produced directly in HBM.  Identical
(seed, device) gives identical bytes.

Workloads (the paper's datasets are not available; these stand in for them):
  paper_example   Sec. 4: X = W [I_r H'] Pi (+ U[0, 1e-3] noise), W and H'
                  uniform on [0, 1], Pi swapping columns i and 10 i for
                  i = 2..r-1, so K = {0, 1, 20, 30, ..., 10 (r-1)}.
  plain_fp64      100,000 x 20, r = 10, W ~ U[0,1), H = I on K and Dirichlet(1)
                  elsewhere, noise max(0, 1e-3 eps); FP64 row-major.
  flow_cytometry  1e7 x 25 (the Sec. 5.2 matrix is 1.6e9 x 25), r = 16,
                  W ~ lognormal(0, 1), Dirichlet(0.5), relative noise
                  max(0, 1e-3 (WH)_ij eps_ij); FP32 row-major.
  flow_kron       the Sec. 5.2 construction X = A (x) A with A p x 5
                  lognormal; R and the column sums have closed forms.
  heat_transfer   5e7 x 64 (the Sec. 5.1 matrix is 4.9e9 x 64), r = 20, W
                  columns are Gaussian bumps over a 1-D index grid, Dirichlet(1),
                  noise max(0, 1e-4 eps); FP32 column-major.
  projection      2e7 x 128, r = 32, W ~ U[0,1), Dirichlet(1), noise
                  max(0, 1e-3 eps); FP32 row-major (BF16 copy by RNE).
  batch           512 matrices, m log-uniform in [1e4, 2e6], n in
                  {16, 32, 64, 128}, r = n / 4, as `projection` otherwise.
"""

import math

import numpy as np
import torch

BASE_SEED = 14026964
CHUNK_ROWS = 1 << 20


def _np_rng(*tag):
    return np.random.default_rng(np.random.SeedSequence([BASE_SEED, *tag]))


def _torch_gen(device, *tag):
    ss = np.random.SeedSequence([BASE_SEED, *tag])
    seed = int(ss.generate_state(1, dtype=np.uint64)[0] & np.uint64(0x7FFFFFFFFFFFFFFF))
    g = torch.Generator(device=device)
    g.manual_seed(seed)
    return g


def planted_h(rng, r, n, alpha):
    """K (sorted, r distinct indices of range(n)) and H (r x n): H(:, K) = I in
    the order of K, other columns Dirichlet(alpha) (nonnegative, sum to one)."""
    K = np.sort(rng.choice(n, size=r, replace=False))
    H = rng.dirichlet(np.full(r, alpha), size=n).T.copy()
    H[:, K] = np.eye(r)
    return [int(k) for k in K], H


def _fill_rows(X_rows_out, m, make_chunk):
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        X_rows_out(i0, i1, make_chunk(i0, i1))


def paper_example(m, noisy=False, r=20, n=200, device="cpu", dtype=torch.float64, seed_tag=0):
    rng = _np_rng(1, seed_tag)
    Hp = rng.uniform(0.0, 1.0, size=(r, n - r))
    B = np.concatenate([np.eye(r), Hp], axis=1)
    perm = np.arange(n)
    for i in range(2, r):
        perm[i], perm[10 * i] = perm[10 * i], perm[i]
    H = B[:, perm]
    K = sorted(int(np.flatnonzero(perm == i)[0]) for i in range(r))
    g = _torch_gen(device, 1, seed_tag, 1)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float64)
    X = torch.empty((m, n), device=device, dtype=dtype)
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        W = torch.rand((i1 - i0, r), generator=g, device=device, dtype=torch.float64)
        C = W @ Ht
        if noisy:
            C += 1e-3 * torch.rand(C.shape, generator=g, device=device, dtype=torch.float64)
        X[i0:i1] = C.to(dtype)
    return {"X": X, "K": K, "H": H, "r": r, "name": "paper_example_noisy" if noisy else "paper_example"}


def plain_fp64(m=100_000, n=20, r=10, device="cpu", seed_tag=0):
    rng = _np_rng(2, seed_tag)
    K, H = planted_h(rng, r, n, 1.0)
    g = _torch_gen(device, 2, seed_tag, 1)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float64)
    X = torch.empty((m, n), device=device, dtype=torch.float64)
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        W = torch.rand((i1 - i0, r), generator=g, device=device, dtype=torch.float64)
        N = torch.clamp(1e-3 * torch.randn((i1 - i0, n), generator=g, device=device, dtype=torch.float64), min=0.0)
        X[i0:i1] = W @ Ht + N
    return {"X": X, "K": K, "H": H, "r": r, "name": f"plain_fp64_{m}x{n}"}


def flow_cytometry(m=10_000_000, n=25, r=16, device="cpu", seed_tag=0):
    rng = _np_rng(3, seed_tag)
    K, H = planted_h(rng, r, n, 0.5)
    g = _torch_gen(device, 3, seed_tag, 1)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float32)
    X = torch.empty((m, n), device=device, dtype=torch.float32)
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        W = torch.exp(torch.randn((i1 - i0, r), generator=g, device=device, dtype=torch.float32))
        WH = W @ Ht
        eps = torch.randn(WH.shape, generator=g, device=device, dtype=torch.float32)
        X[i0:i1] = WH + torch.clamp(1e-3 * WH * eps, min=0.0)
    return {"X": X, "K": K, "H": H, "r": r, "name": f"flow_cytometry_{m}x{n}"}


def kron_factor(p, q=5, seed_tag=0):
    """A (p x q) lognormal(0, 1) in FP32, the factor of X = A (x) A."""
    rng = _np_rng(4, seed_tag)
    return np.exp(rng.standard_normal((p, q))).astype(np.float32)


def flow_kron(p=3162, q=5, device="cpu", seed_tag=0):
    """X = A (x) A (row i*p + i', column a*q + b holds A[i, a] A[i', b]).  The
    product of two FP32 numbers is rounded to FP32 once; the closed forms are
    checked against the rounded bytes only through their invariants."""
    A = kron_factor(p, q, seed_tag)
    At = torch.from_numpy(A).to(device)
    X = torch.kron(At, At).contiguous()
    return {"X": X, "A": A, "name": f"flow_kron_{p*p}x{q*q}"}


def heat_transfer(m=50_000_000, n=64, r=20, device="cpu", seed_tag=0, col_major=True):
    """Returns X with X["X"] of shape (m, n); when col_major it is a transposed
    view of an (n, m) contiguous tensor, i.e. column-major with ld = m."""
    rng = _np_rng(5, seed_tag)
    K, H = planted_h(rng, r, n, 1.0)
    centres = rng.uniform(0.0, 1.0, size=r)
    widths = rng.uniform(0.005, 0.05, size=r)
    g = _torch_gen(device, 5, seed_tag, 1)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float32)
    c = torch.from_numpy(centres).to(device=device, dtype=torch.float64)
    w = torch.from_numpy(widths).to(device=device, dtype=torch.float64)
    store = torch.empty((n, m) if col_major else (m, n), device=device, dtype=torch.float32)
    denom = float(max(m - 1, 1))
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        t = torch.arange(i0, i1, device=device, dtype=torch.float64) / denom
        W = torch.exp(-((t[:, None] - c[None, :]) ** 2) / (2.0 * w[None, :] ** 2)).to(torch.float32)
        C = W @ Ht + torch.clamp(1e-4 * torch.randn((i1 - i0, n), generator=g, device=device, dtype=torch.float32), min=0.0)
        if col_major:
            store[:, i0:i1] = C.T
        else:
            store[i0:i1] = C
    X = store.T if col_major else store
    return {"X": X, "K": K, "H": H, "r": r, "name": f"heat_transfer_{m}x{n}", "col_major": col_major}


def projection(m=20_000_000, n=128, r=32, device="cpu", seed_tag=0):
    rng = _np_rng(6, seed_tag)
    K, H = planted_h(rng, r, n, 1.0)
    g = _torch_gen(device, 6, seed_tag, 1)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float32)
    X = torch.empty((m, n), device=device, dtype=torch.float32)
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        W = torch.rand((i1 - i0, r), generator=g, device=device, dtype=torch.float32)
        X[i0:i1] = W @ Ht + torch.clamp(1e-3 * torch.randn((i1 - i0, n), generator=g, device=device, dtype=torch.float32), min=0.0)
    return {"X": X, "K": K, "H": H, "r": r, "name": f"projection_{m}x{n}"}


def batch_shapes(count=512, m_lo=10_000, m_hi=2_000_000, ns=(16, 32, 64, 128), seed_tag=0):
    rng = _np_rng(7, seed_tag)
    ms = np.rint(np.exp(rng.uniform(math.log(m_lo), math.log(m_hi), size=count))).astype(np.int64)
    nn = rng.choice(np.asarray(ns), size=count)
    return [(int(a), int(b)) for a, b in zip(ms, nn)]


def batch_matrix(idx, m, n, device="cpu", seed_tag=0):
    r = max(1, n // 4)
    rng = _np_rng(8, seed_tag, idx)
    K, H = planted_h(rng, r, n, 1.0)
    g = _torch_gen(device, 8, seed_tag, idx)
    Ht = torch.from_numpy(H).to(device=device, dtype=torch.float32)
    X = torch.empty((m, n), device=device, dtype=torch.float32)
    for i0 in range(0, m, CHUNK_ROWS):
        i1 = min(m, i0 + CHUNK_ROWS)
        W = torch.rand((i1 - i0, r), generator=g, device=device, dtype=torch.float32)
        X[i0:i1] = W @ Ht + torch.clamp(1e-3 * torch.randn((i1 - i0, n), generator=g, device=device, dtype=torch.float32), min=0.0)
    return {"X": X, "K": K, "H": H, "r": r, "name": f"batch_{idx}_{m}x{n}"}


def random_matrix(m, n, device="cpu", dtype=torch.float32, seed_tag=0, dist="uniform"):
    """Plain random test matrices (edge cases, tiny shapes)."""
    g = _torch_gen(device, 9, seed_tag, m, n)
    if dist == "uniform":
        X = torch.rand((m, n), generator=g, device=device, dtype=torch.float64)
    elif dist == "normal":
        X = torch.randn((m, n), generator=g, device=device, dtype=torch.float64)
    elif dist == "lognormal":
        X = torch.exp(torch.randn((m, n), generator=g, device=device, dtype=torch.float64))
    else:
        raise ValueError(dist)
    return X.to(dtype)
