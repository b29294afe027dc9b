"""Pins for the oracle's small dense factorizations (eq. 6 thin QR, eq. 8 QRCP)
against LAPACK (scipy's dgeqrf / dgeqp3), numpy's SVD and invariants."""
import numpy as np
import pytest
import scipy.linalg as sl
from scipy.linalg import lapack

from oracle.dense import householder_qr, jacobi_svd, qrcp


@pytest.mark.parametrize("m,l", [(50, 50), (300, 17), (1000, 64), (129, 128)])
def test_householder_qr_vs_dgeqrf(m, l):
    X = np.random.default_rng(m + l).standard_normal((m, l))
    Q, R = householder_qr(X)
    assert np.max(np.abs(Q.T @ Q - np.eye(l))) < 5e-15 * np.sqrt(m)
    assert np.max(np.abs(Q @ R - X)) < 1e-14 * np.abs(X).max() * np.sqrt(m)
    assert np.all(np.diag(R) >= 0)
    assert np.all(np.tril(R, -1) == 0)
    qr, tau, work, info = lapack.dgeqrf(X)
    Rl = np.triu(qr[:l, :])
    s = np.sign(np.diag(Rl))
    np.testing.assert_allclose(R, s[:, None] * Rl, rtol=0, atol=1e-12 * np.abs(Rl).max())


def test_householder_qr_rank_deficient_stays_orthonormal():
    rng = np.random.default_rng(3)
    X = rng.standard_normal((200, 5)) @ rng.standard_normal((5, 12))
    X[:, 7] = 0.0
    Q, R = householder_qr(X)
    assert np.max(np.abs(Q.T @ Q - np.eye(12))) < 1e-13
    assert np.max(np.abs(Q @ R - X)) < 1e-12 * np.abs(X).max()


@pytest.mark.parametrize("l", [8, 40, 110])
def test_qrcp_vs_dgeqp3_separated_norms(l):
    rng = np.random.default_rng(l)
    # well separated column norms so that both pivot sequences are forced
    D = rng.standard_normal((l, l)) * np.logspace(0, -6, l)[rng.permutation(l)]
    Qt, R, piv = qrcp(D)
    Qs, Rs, Ps = sl.qr(D, pivoting=True)
    np.testing.assert_array_equal(piv, Ps)
    s = np.sign(np.diag(Rs))
    np.testing.assert_allclose(R, s[:, None] * Rs, rtol=0, atol=1e-13 * np.abs(D).max())
    assert np.max(np.abs(Qt.T @ Qt - np.eye(l))) < 1e-14 * l
    assert np.max(np.abs(Qt @ R - D[:, piv])) < 1e-14 * l * np.abs(D).max()


def test_qrcp_invariants_and_rank_revealing():
    rng = np.random.default_rng(7)
    l = 60
    D = rng.standard_normal((l, 10)) @ rng.standard_normal((10, l)) + 1e-9 * rng.standard_normal((l, l))
    Qt, R, piv = qrcp(D)
    d = np.diag(R)
    assert np.all(d >= 0)
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))  # non-increasing diagonal
    assert np.all(np.tril(R, -1) == 0)
    assert sorted(piv.tolist()) == list(range(l))
    assert d[9] / d[10] > 1e5  # the rank-10 gap is revealed
    # prod |R_ii| = |det D| = prod sigma_i, on a well-conditioned matrix
    G = rng.standard_normal((l, l)) + 4 * np.eye(l)
    dg = np.diag(qrcp(G)[1])
    assert np.prod(dg / np.linalg.svd(G, compute_uv=False)) == pytest.approx(1.0, rel=1e-11)


def test_qrcp_ties_and_zero_columns():
    # two identical columns of largest norm: the lower position wins
    D = np.zeros((4, 4))
    D[:, 1] = [1, 2, 3, 4]
    D[:, 3] = [1, 2, 3, 4]
    D[0, 2] = 0.5
    Qt, R, piv = qrcp(D)
    assert piv[0] == 1
    np.testing.assert_allclose(Qt @ R, D[:, piv], atol=1e-14)
    Z = np.zeros((5, 5))
    Qt, R, piv = qrcp(Z)
    np.testing.assert_array_equal(piv, np.arange(5))
    np.testing.assert_array_equal(Qt, np.eye(5))
    assert np.all(R == 0)


def test_qrcp_is_deterministic_bitwise():
    D = np.random.default_rng(11).standard_normal((33, 33))
    a = qrcp(D)
    b = qrcp(D.copy())
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)


@pytest.mark.parametrize("m,n", [(40, 40), (120, 30), (30, 90)])
def test_jacobi_svd_vs_numpy(m, n):
    A = np.random.default_rng(m * n).standard_normal((m, n))
    U, s, V = jacobi_svd(A)
    ref = np.linalg.svd(A, compute_uv=False)
    np.testing.assert_allclose(s, ref, rtol=1e-12, atol=1e-13 * ref[0])
    np.testing.assert_allclose(U @ np.diag(s) @ V.T, A, atol=1e-12 * ref[0])


def test_qrcp_replay_of_its_own_pivots_is_bit_identical():
    """follow= with the oracle's own pivots changes nothing, and the trace
    shows the argmax chosen at every step."""
    D = np.random.default_rng(13).standard_normal((37, 37)) * np.logspace(0, -5, 37)
    a = qrcp(D)
    trace = []
    b = qrcp(D, follow=a[2], trace=trace)
    for x, y in zip(a, b):
        np.testing.assert_array_equal(x, y)
    assert len(trace) == 37
    assert all(int(np.argmax(acc)) == c for acc, c in trace)
    with pytest.raises(ValueError):
        qrcp(D, follow=np.zeros(37, dtype=np.int32))


def test_qrcp_replay_of_other_pivots_is_still_a_factorization():
    """Any pivot sequence gives D[:, piv] = Qt R with orthogonal Qt."""
    rng = np.random.default_rng(14)
    D = rng.standard_normal((20, 20))
    order = rng.permutation(20).astype(np.int32)
    Qt, R, piv = qrcp(D, follow=order)
    np.testing.assert_array_equal(piv, order)
    assert np.max(np.abs(Qt @ R - D[:, piv])) < 1e-13
    assert np.max(np.abs(Qt.T @ Qt - np.eye(20))) < 1e-14


def test_pivot_margin_rule_accepts_rounding_and_catches_wrong_pivots():
    """The margin rule used to compare QRCP implementations: a QRCP whose
    norms are summed in another order (here: reversed row order, the same
    factorization otherwise) passes, listing at most a few near-tie steps; a
    sequence with two decided pivots exchanged, or ordered by smallest norm,
    fails."""
    from tests.pivots import margin_tau, pivot_margins

    rng = np.random.default_rng(15)
    l = 60
    D = rng.standard_normal((l, l)) * np.logspace(0, -8, l)[rng.permutation(l)]
    tau = margin_tau(D)
    # reversed summation order: the oracle on the row-reversed matrix sums
    # every column norm in the opposite order and has the same pivots up to
    # rounding (a row permutation leaves column norms unchanged)
    piv_rev = qrcp(D[::-1].copy())[2]
    near = pivot_margins(D, piv_rev, tau)
    assert len(near) <= 2
    piv = qrcp(D)[2]
    bad = piv.copy()
    bad[[3, 4]] = bad[[4, 3]]
    with pytest.raises(AssertionError):
        pivot_margins(D, bad, tau)
    worst = np.argsort(np.linalg.norm(D, axis=0)).astype(np.int32)
    with pytest.raises(AssertionError):
        pivot_margins(D, worst, tau)
