"""CPU oracle for the single-pass TSQR / Gaussian-projection NMF path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may use it.  It is a plain, slow, obviously-correct FP64 restatement
of what the method computes (Benson, Lee, Rajwa, Gleich, "Scalable methods for
nonnegative matrix factorizations of near-separable tall-and-skinny matrices"),
written with numpy and shares no code, table or helper with the HIP library.

Modules
    tsqr        thin-QR R factor by Householder leaves + a binary tree (Sec. 3.1),
                sign finalisation, reference column sums / Gram (Sec. 3.3).
    select      SPA and greedy XRAY on the reduced matrix (Sec. 2.1, 2.2),
                Gaussian-projection selection (Sec. 2.3).
    nnls        Lawson-Hanson nonnegative least squares for H (Sec. 2.4).
    residual    relative residual in the reduced space (Sec. 2.4, Sec. 4).
    philox      Philox4x32-10 counter-based generator + Box-Muller normals,
                restated from Salmon et al. (SC'11), used as G of Sec. 2.3.
    gauss_proj  Y = G^T X accumulated row by row (Algorithm 1, Sec. 3.2).
    rsvd        singular values and vectors of R (Sec. 3.1, R-SVD) and the
                residual curve over candidate ranks r (Sec. 2.2, Sec. 2.4).
    parallel    the same leaf factors and tree, with runs of leaves in worker
                processes (used to time the oracle on every host core).

Pins: every function is checked in ``tests/test_oracle_*.py`` against facts the
paper and the mathematics fix (LAPACK on tiny inputs, closed forms such as the
Kronecker and tiled-copy R factors, planted extreme columns, scipy's NNLS plus
KKT conditions, rocRAND's Philox rounds).  No function here is "parity
unpinned".
"""

from . import tsqr, select, nnls, residual, philox, gauss_proj, rsvd  # noqa: F401
