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
