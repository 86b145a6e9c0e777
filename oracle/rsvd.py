"""Oracle: SVD of the n x n factor R, and the rank sweep (test infrastructure).

Sec. 3.1 (TSQR and R-SVD): with X = QR and R = U S V^T, X = (QU) S V^T is the
SVD of X, so its singular values and right singular vectors come from the
small R.  Sec. 2.2 and Sec. 2.4: the selection, the NNLS fit and the
residual can all be computed on R, so residuals for many candidate ranks r
cost only n x n work -- the residual curves of the paper's figures.

  rsvd        singular values (descending) and V of R, with U; each pair
              (u_i, v_i) signed so that the largest-magnitude entry of v_i
              is positive (singular vectors are unique up to that sign when
              the singular values are distinct).  The decomposition itself is
              LAPACK's (numpy.linalg.svd), a library primitive.
  rank_sweep  SPA with rmax picks on R D^{-1}; for r = 1..rmax the NNLS fit
              of R on its first r picked columns and the relative residual.
"""

import numpy as np

from . import nnls as _nnls
from . import residual as _res
from . import select as _sel


def sign_fix(U, V):
    """Flip (u_i, v_i) so that the largest-magnitude entry of v_i is positive."""
    U = np.array(U, copy=True)
    V = np.array(V, copy=True)
    for i in range(V.shape[1]):
        j = int(np.argmax(np.abs(V[:, i])))
        if V[j, i] < 0:
            V[:, i] = -V[:, i]
            U[:, i] = -U[:, i]
    return U, V


def rsvd(R):
    """(s, U, V) with R = U diag(s) V^T, s descending."""
    R = np.asarray(R, dtype=np.float64)
    U, s, Vt = np.linalg.svd(R)
    U, V = sign_fix(U, Vt.T)
    return s, U, V


def rank_sweep(R, rmax, colscale=None):
    """(K, resid): K the SPA picks (rmax of them, in order) and resid[r - 1] the
    relative residual ||R - R(:, K[:r]) H_r||_F^2 / ||R||_F^2 of the NNLS fit
    on the first r picks."""
    R = np.asarray(R, dtype=np.float64)
    K, _, got = _sel.spa(R, rmax, colscale=colscale)
    resid = []
    for r in range(1, got + 1):
        H, _, _ = _nnls.nnls_matrix(R, K[:r])
        resid.append(_res.relative_residual(R, K[:r], H))
    return K, np.asarray(resid)
