"""Oracle: the Gaussian matrix G of the projection, as a fixed function of
(seed, row, column) (test infrastructure).

Sec. 2.3 uses G in R^{m x k} with i.i.d. N(0, 1) entries, and Sec. 3.2
(Algorithm 1) samples the row g_i next to the data row x_i.  Sec. 3.2 also
notes that independently seeded generators on different processors may be
slightly correlated; a counter-based generator keyed by the global row index
avoids that and makes G independent of how rows are split among workers.

Generator: Philox4x32 with 10 rounds, restated from its published definition
(J. Salmon, M. Moraes, R. Dror, D. Shaw, "Parallel random numbers: as easy as
1, 2, 3", SC'11).  One round maps the counter (c0, c1, c2, c3) under key
(k0, k1) to
    (hi(M1*c2) ^ c1 ^ k0,  lo(M1*c2),  hi(M0*c0) ^ c3 ^ k1,  lo(M0*c0)),
with 32x32->64-bit products split into high and low words; between rounds the
key is advanced by the Weyl increments (W0, W1).  The multipliers and
increments below are the ones that paper specifies for Philox4x32.

Mapping to G (the library's contract, restated independently on the device):
    key     = (seed mod 2^32, seed >> 32)
    counter = (i mod 2^32, i >> 32, q, 0)        for row i, column group q
    (x0, x1, x2, x3) = Philox4x32-10(counter, key)
    u_a     = ((x_a >> 8) + 1) * 2^-24           in (0, 1], exact in FP32
    G[i, 4q + 0], G[i, 4q + 1] = sqrt(-2 ln u0) * (cos 2 pi u1, sin 2 pi u1)
    G[i, 4q + 2], G[i, 4q + 3] = sqrt(-2 ln u2) * (cos 2 pi u3, sin 2 pi u3)
(Box-Muller, 1958.)
"""

import numpy as np

PHILOX_M0 = 0xD2511F53
PHILOX_M1 = 0xCD9E8D57
PHILOX_W0 = 0x9E3779B9
PHILOX_W1 = 0xBB67AE85
_MASK = np.uint64(0xFFFFFFFF)


def philox4x32_10(c0, c1, c2, c3, k0, k1):
    """Vectorised Philox4x32-10.  Counter words are arrays (or scalars) of
    uint32 values; the key is two Python ints.  Returns four uint32 arrays."""
    c0 = np.asarray(c0, dtype=np.uint64) & _MASK
    c1 = np.asarray(c1, dtype=np.uint64) & _MASK
    c2 = np.asarray(c2, dtype=np.uint64) & _MASK
    c3 = np.asarray(c3, dtype=np.uint64) & _MASK
    k0 = int(k0) & 0xFFFFFFFF
    k1 = int(k1) & 0xFFFFFFFF
    m0 = np.uint64(PHILOX_M0)
    m1 = np.uint64(PHILOX_M1)
    for rnd in range(10):
        p0 = m0 * c0                      # < 2^64, exact in uint64
        p1 = m1 * c2
        hi0, lo0 = p0 >> np.uint64(32), p0 & _MASK
        hi1, lo1 = p1 >> np.uint64(32), p1 & _MASK
        c0, c1, c2, c3 = (hi1 ^ c1 ^ np.uint64(k0), lo1,
                          hi0 ^ c3 ^ np.uint64(k1), lo0)
        if rnd < 9:
            k0 = (k0 + PHILOX_W0) & 0xFFFFFFFF
            k1 = (k1 + PHILOX_W1) & 0xFFFFFFFF
    return (c0.astype(np.uint32), c1.astype(np.uint32),
            c2.astype(np.uint32), c3.astype(np.uint32))


def uniform_open0(x):
    """u = ((x >> 8) + 1) * 2^-24 in (0, 1] (never 0, so log(u) is finite)."""
    x = np.asarray(x, dtype=np.uint64)
    return ((x >> np.uint64(8)) + np.uint64(1)).astype(np.float64) * 2.0 ** -24


def box_muller(ua, ub):
    """Two independent N(0, 1) values from two uniforms in (0, 1]."""
    rad = np.sqrt(-2.0 * np.log(ua))
    ang = 2.0 * np.pi * ub
    return rad * np.cos(ang), rad * np.sin(ang)


def gaussian_block(seed, rows, q):
    """G[rows, 4q:4q+4] as an (len(rows), 4) FP64 array."""
    rows = np.asarray(rows, dtype=np.uint64)
    seed = int(seed)
    x0, x1, x2, x3 = philox4x32_10(rows & _MASK, rows >> np.uint64(32),
                                   np.full(rows.shape, q, dtype=np.uint64),
                                   np.zeros(rows.shape, dtype=np.uint64),
                                   seed & 0xFFFFFFFF, seed >> 32)
    g0, g1 = box_muller(uniform_open0(x0), uniform_open0(x1))
    g2, g3 = box_muller(uniform_open0(x2), uniform_open0(x3))
    return np.stack([g0, g1, g2, g3], axis=1)


def gaussian_matrix(seed, row0, nrows, k):
    """G[row0:row0+nrows, 0:k] (k a multiple of 4) in FP64."""
    if k % 4 != 0:
        raise ValueError("k must be a multiple of 4")
    rows = np.arange(row0, row0 + nrows, dtype=np.uint64)
    return np.concatenate([gaussian_block(seed, rows, q) for q in range(k // 4)], axis=1)
