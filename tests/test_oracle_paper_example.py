"""P16: the synthetic experiment of Sec. 4 at reduced m.

The paper builds X = W [I_r H'] Pi with m = 2e8, n = 200, r = 20, W and H'
uniform on [0, 1], Pi swapping columns i and 10 i for i = 2..19, and reports
that SPA and GP recover all 20 extreme columns at r = 20 with the relative
residual reaching zero, that greedy XRAY needs 21 picks to contain them, and
that adding U[0, 1e-3] noise changes nothing.  The same recipe is run here with
m = 20,000 rows; the statements do not depend on m.
"""

import numpy as np
import pytest
import torch

from oracle import gauss_proj, nnls, residual, select, tsqr
from paper_1402_6964_amd import synth

import os


def _golden():
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "sec4_synthetic_example.txt")
    out = {}
    with open(path) as fh:
        for line in fh:
            if line.strip() and not line.startswith("#"):
                k, *v = line.split()
                out[k] = v
    return out


GOLDEN = _golden()
PLANTED = [int(v) for v in GOLDEN["extreme"]]
XRAY_PICKS = int(GOLDEN["xray_picks_containing_all"][0])


@pytest.fixture(scope="module", params=[False, True], ids=["exact", "noisy"])
def example(request):
    d = synth.paper_example(20_000, noisy=request.param, device="cpu", dtype=torch.float64)
    X = d["X"].numpy()
    R = tsqr.tsqr_r_final(X, leaf_rows=1000)
    colsum, _, gram = tsqr.reference_sums(X)
    return {"X": X, "R": R, "d": colsum, "K": d["K"], "noisy": request.param}


def test_planted_set_follows_the_swap_rule(example):
    """The generator's extreme set is the one the swap rule of Sec. 4 gives."""
    r = int(GOLDEN["r"][0])
    lo, hi = int(GOLDEN["swap_first"][0]), int(GOLDEN["swap_last"][0])
    perm = list(range(int(GOLDEN["n"][0])))
    for i in range(lo, hi + 1):
        perm[i], perm[10 * i] = perm[10 * i], perm[i]
    assert sorted(perm.index(j) for j in range(r)) == PLANTED
    assert example["K"] == PLANTED and len(PLANTED) == r


def test_spa_recovers_all_extreme_columns(example):
    K, _, info = select.spa(example["R"], 20, colscale=example["d"])
    assert sorted(K) == PLANTED and info == 20


def test_gp_recovers_all_extreme_columns(example):
    Y = gauss_proj.gauss_proj(example["X"], 128, 14026964)
    K, counts, info = select.gp_select(Y, 20, colscale=example["d"])
    assert sorted(K) == PLANTED


def test_residual_vanishes_at_r20(example):
    R = example["R"]
    H, _, _ = nnls.nnls_matrix(R, PLANTED)
    rho = residual.relative_residual(R, PLANTED, H)
    if example["noisy"]:
        assert rho < 1e-6
    else:
        assert rho < 1e-20
        cols = list(range(0, 200, 23))
        Hx, rx, _ = nnls.nnls_matrix(example["X"], PLANTED, cols=cols)
        assert np.abs(Hx[:, cols] - H[:, cols]).max() < 1e-10
        assert np.all(rx[cols] < 1e-18 * np.sum(example["X"] ** 2))
    H19, _, _ = nnls.nnls_matrix(R, PLANTED[:19])
    assert residual.relative_residual(R, PLANTED[:19], H19) > 1e-4


@pytest.mark.slow
def test_xray_first_21_picks_contain_the_extreme_columns(example):
    """The Fig. 2 caption and the Sec. 4 text disagree on XRAY; the text says
    the first 21 greedy picks contain all 20 extreme columns, and so they do."""
    K, _ = select.xray(example["R"], XRAY_PICKS)
    assert set(PLANTED) <= set(K)
