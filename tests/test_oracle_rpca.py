"""Pins for the ALM-CoRUTV oracle (Sec. 4, Algorithm 2; Sec. 5.3, Table 1).

* the shrinkage operator against its closed form;
* Table 1's printed outcomes (golden fixture with citation): exact rank and
  exact support recovery, relative residual below the stopping threshold, and
  an iteration count near the printed 12 (mu_0 and rho are not printed, so the
  count is only loosely pinned);
* the robust-PCA workload at the video-frames shape (tall, rank 5, 5 % uniform
  corruptions) at reduced height: exact support recovery and ||L - L*|| small.
"""
import json
import os

import numpy as np
import pytest

from oracle.rpca import alm_corutv, shrink, threshold_rank
from workloads import low_rank_plus_sparse

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "table1_rpca.json")


def test_shrink_closed_form():
    x = np.array([-3.0, -1.0, -0.5, 0.0, 0.25, 1.0, 2.5])
    np.testing.assert_array_equal(shrink(x, 1.0), [-2.0, 0.0, 0.0, 0.0, 0.0, 0.0, 1.5])
    assert np.all(shrink(x, 0.0) == x)


def test_threshold_rank_counts_diagonal_entries_above_delta():
    """eq. 12 keeps the diagonal entries of T greater than delta (strictly);
    the count is taken over the whole diagonal, which for the non-increasing
    diagonal of a QRCP is a prefix."""
    T = np.diag([5.0, 3.0, 1.0, 1.0, 0.5])
    assert threshold_rank(T, 1.0) == 2
    assert threshold_rank(T, 0.4) == 5
    assert threshold_rank(T, 9.0) == 0
    # a diagonal that rounding left out of order: every entry above delta counts
    assert threshold_rank(np.diag([5.0, 1.0, 3.0]), 2.0) == 2


def _rows():
    with open(GOLDEN) as f:
        g = json.load(f)
    return g["rows"], g["stop_tol"]


@pytest.mark.parametrize("n", [1000, pytest.param(2000, marks=pytest.mark.slow)])
def test_table1_exact_recovery(n):
    rows, tol = _rows()
    row = next(r for r in rows if r["n"] == n)
    k = row["rank_L"]
    M, L, S = low_rank_plus_sparse(n, n, k, row["nnz_S"] / n**2, 80.0, seed=n, values="pm")
    assert np.count_nonzero(S) == row["nnz_S"]
    Lh, Sh, info = alm_corutv(M, k, k, 1, seed=7, max_iter=60, tol=tol)  # l = 2k, q = 1
    assert np.linalg.matrix_rank(Lh) == row["rank_Lstar"]
    assert np.count_nonzero(Sh) == row["nnz_Sstar"]
    assert np.array_equal(Sh != 0, S != 0)
    assert info["zeta"] < tol
    assert abs(info["iters"] - row["iters"]) <= 4


def test_frames_shaped_rpca_recovers_support():
    m, n = 7680, 300
    M, L, S = low_rank_plus_sparse(m, n, 5, 0.05, 50.0, seed=4)
    Lh, Sh, info = alm_corutv(M, 5, 5, 1, seed=4, max_iter=50)
    assert info["lam"] == pytest.approx(1 / np.sqrt(m))
    assert np.linalg.norm(Lh - L) / np.linalg.norm(L) <= 1e-5
    # support: the exact nonzeros of S* equal the planted ones
    assert np.array_equal(Sh != 0, S != 0)
    assert info["ranks"][-1] == 5


@pytest.mark.parametrize("m,n", [(120, 3000), (900, 1300)])
def test_wide_input_is_the_transposed_problem(m, n):
    """A wide M runs CoR-UTV on the transposed problem (lower T, Sec. 3), and
    its thresholding keeps the columns of T (eq. 12 on the transposed
    problem).  Every operator of Algorithm 2 commutes with transposition, so
    the run on M^T equals the transposed run on M, up to the rounding of
    associating the rank-r products differently."""
    Mw, L, S = low_rank_plus_sparse(m, n, 4, 0.05, 20.0, seed=m + n)
    a_L, a_S, a = alm_corutv(Mw, 4, 4, 1, seed=3, max_iter=25)
    b_L, b_S, b = alm_corutv(Mw.T.copy(), 4, 4, 1, seed=3, max_iter=25)
    assert a["ranks"] == b["ranks"]
    assert np.array_equal(a_S != 0, b_S.T != 0)
    nL = np.linalg.norm(b_L)
    assert np.linalg.norm(a_L - b_L.T) <= 1e-12 * nL
    assert np.linalg.norm(a_S - b_S.T) <= 1e-12 * nL
