"""Pins for the CoR-UTV oracle (Sec. 3, eqs. 4-9, Algorithm 1; Sec. 5.1-5.2).

Each test ties the oracle to something other than itself: exact recovery of an
exactly low-rank matrix, orthonormality and triangularity, the range-finder
closed form computed through LAPACK, the identity D = R_Z^T, the literal
Algorithm 1, Eckart-Young via the Jacobi SVD and the published average-case
bound of the randomized range finder, and the qualitative claims of Sec. 5.
"""
import numpy as np
import pytest

from oracle.corutv import corutv, rel_err, truncate
from oracle.dense import jacobi_svd
from workloads import decaying, noisy_low_rank, sec51_matrix

U_EPS = np.finfo(np.float64).eps


@pytest.mark.parametrize("m,n,k,p,q,tri", [
    (300, 200, 10, 5, 0, "auto"), (300, 200, 10, 5, 1, "upper"), (300, 200, 10, 6, 2, "lower"),
    (150, 400, 7, 3, 1, "auto"), (150, 400, 7, 3, 0, "upper"), (257, 129, 20, 0, 1, "auto"),
])
def test_exact_rank_k_is_recovered(m, n, k, p, q, tri):
    """P1: for rank(A) = k <= l the range of Q1 contains range(A), so U T V^T = A."""
    A = noisy_low_rank(m, n, k, 0.0, seed=m + n + k)
    r = corutv(A, k, p, q, seed=3, tri=tri)
    assert rel_err(A, r["U"], r["T"], r["V"]) <= 1e-12
    ell = k + p
    assert r["U"].shape == (m, ell) and r["V"].shape == (n, ell) and r["T"].shape == (ell, ell)


@pytest.mark.parametrize("m,n,tri", [(400, 300, "upper"), (400, 300, "lower"), (200, 500, "auto")])
def test_orthonormal_and_triangular(m, n, tri):
    """P2/P3: U, V orthonormal to 1e-13; T exactly triangular; diag(T) >= 0 and non-increasing."""
    A = decaying(m, n, 60, 1e-4, seed=9)
    r = corutv(A, 20, 10, 1, seed=4, tri=tri)
    ell = 30
    assert np.max(np.abs(r["U"].T @ r["U"] - np.eye(ell))) <= 1e-13
    assert np.max(np.abs(r["V"].T @ r["V"] - np.eye(ell))) <= 1e-13
    T = r["T"]
    lower = (tri == "lower") or (tri == "auto" and m < n)
    if lower:
        assert np.all(np.triu(T, 1) == 0)
    else:
        assert np.all(np.tril(T, -1) == 0)
    d = np.diag(T)
    assert np.all(d >= 0)
    assert np.all(d[:-1] >= d[1:] * (1 - 1e-12))


@pytest.mark.parametrize("q", [0, 1])
def test_range_finder_closed_form_via_lapack(q):
    """P4: U T V^T = Q Q^T A with Q an orthonormal basis of A (A^T A)^q Psi,
    here obtained by LAPACK's QR of the literal sketch (an independent route)."""
    A = decaying(250, 180, 40, 1e-3, seed=21, kind="poly", alpha=0.5)
    r = corutv(A, 12, 8, q, seed=8)
    C1 = A @ r["Omega"]
    for _ in range(q):
        C1 = A @ (A.T @ C1)
    Q, _ = np.linalg.qr(C1)
    ref = Q @ (Q.T @ A)
    got = r["U"] @ r["T"] @ r["V"].T
    assert np.linalg.norm(got - ref) <= 1e-12 * np.linalg.norm(A)


def test_core_equals_transposed_R_of_Z():
    """P5: D = Q1^T A Q2 = (A^T Q1)^T Q2 = R_Z^T, so D is lower triangular."""
    A = decaying(300, 220, 80, 1e-3, seed=5)
    r = corutv(A, 25, 10, 1, seed=2)
    D, RZ = r["D"], r["R_Z"]
    scale = np.linalg.norm(A, 2)
    assert np.linalg.norm(np.triu(D, 1)) <= 1e-13 * scale * D.shape[0]
    assert np.linalg.norm(D - RZ.T) <= 1e-13 * scale * D.shape[0]


@pytest.mark.parametrize("q", [0, 1, 2])
def test_literal_algorithm1_equals_stabilized(q):
    """P6: the literal Algorithm 1 (no re-orthonormalisation inside the power
    loop) and the re-orthonormalised loop give the same Q1, Q2 and output on a
    well-conditioned input (condition number of the sketch ~ (s1/sl)^(2q+1))."""
    rng = np.random.default_rng(31)
    m, n, ell = 120, 90, 12
    U0 = np.linalg.qr(rng.standard_normal((m, ell)))[0]
    V0 = np.linalg.qr(rng.standard_normal((n, ell)))[0]
    A = (U0 * np.linspace(2.0, 1.0, ell)) @ V0.T + 1e-3 * rng.standard_normal((m, n))
    lit = corutv(A, 8, 4, q, seed=6, mode="literal")
    st = corutv(A, 8, 4, q, seed=6)
    tol = 1e-12 * 4.0 ** (2 * q + 1)
    assert np.max(np.abs(lit["Q1"] - st["Q1"])) < tol
    assert np.max(np.abs(lit["Q2"] - st["Q2"])) < tol
    np.testing.assert_array_equal(lit["piv"], st["piv"])
    assert np.max(np.abs(lit["T"] - st["T"])) < tol * 10


def test_interlacing_and_determinant():
    """P7: sigma(T) = sigma(D) <= sigma(A) (D is a compression of A) and
    prod |T_ii| = prod sigma_i(D), with singular values from the Jacobi SVD."""
    A = decaying(160, 120, 50, 1e-2, seed=12, kind="poly", alpha=1.0)
    r = corutv(A, 15, 5, 1, seed=1)
    sT = jacobi_svd(r["T"])[1]
    sD = jacobi_svd(r["D"])[1]
    sA = jacobi_svd(A)[1]
    np.testing.assert_allclose(sT, sD, rtol=1e-11, atol=1e-14 * sA[0])
    assert np.all(sD <= sA[:20] * (1 + 1e-12))
    assert np.prod(np.diag(r["T"]) / sD) == pytest.approx(1.0, rel=1e-9)


def test_eckart_young_and_average_case_bound():
    """P8: e_l >= optimal rank-l error (Eckart-Young, eq. 3), and over 20 draws
    (Sec. 5.1 averages 20 trials) the mean error obeys the randomized range
    finder's average Frobenius bound sqrt(1 + k/(p-1)) ||A - A_k||_F, which
    applies because U T V^T = Q1 Q1^T A."""
    A = decaying(200, 150, 150, 0.0, seed=40, kind="poly", alpha=1.0)
    s = jacobi_svd(A)[1]
    k, p = 10, 6
    ell = k + p
    opt_l = np.sqrt(np.sum(s[ell:] ** 2))
    opt_k = np.sqrt(np.sum(s[k:] ** 2))
    errs = []
    for seed in range(20):
        r = corutv(A, k, p, 0, seed=seed)
        e = np.linalg.norm(A - r["U"] @ r["T"] @ r["V"].T)
        assert e >= opt_l * (1 - 1e-12)
        errs.append(e)
    assert np.mean(errs) <= np.sqrt(1 + k / (p - 1)) * opt_k * 1.1


def test_rank_revealing_gap_and_threshold_rank():
    """P9: rank-k plus eps noise: T_{k+1,k+1} / T_kk is of the order of the
    noise, and counting diagonals above a threshold inside the gap gives k."""
    A = noisy_low_rank(300, 250, 12, 1e-8, seed=17)
    r = corutv(A, 12, 8, 1, seed=5)
    d = np.diag(r["T"])
    # noise spectral norm ~ 1e-8 (sqrt(m) + sqrt(n)) ~ 3e-7 against a signal
    # sigma_k of order 10: the ratio sits near 1e-8, far below 1e-6
    assert d[12] / d[11] < 1e-6
    delta = np.sqrt(d[11] * d[12])
    assert int(np.sum(d > delta)) == 12


def test_full_sample_size_is_an_exact_factorization():
    """P10: l = min(m, n) makes Q2 square orthogonal, so A = U T V^T exactly."""
    A = np.random.default_rng(2).standard_normal((90, 40))
    r = corutv(A, 30, 10, 1, seed=3)
    assert rel_err(A, r["U"], r["T"], r["V"]) <= 50 * U_EPS


def test_wide_matrix_is_the_transposed_problem():
    """P13: for m < n the output is the transpose-swap of the tall problem."""
    A = decaying(120, 300, 40, 1e-4, seed=8)
    a = corutv(A, 10, 5, 1, seed=9)
    b = corutv(A.T.copy(), 10, 5, 1, seed=9, tri="upper")
    np.testing.assert_array_equal(a["U"], b["V"])
    np.testing.assert_array_equal(a["V"], b["U"])
    np.testing.assert_array_equal(a["T"], b["T"].T)
    assert np.all(np.triu(a["T"], 1) == 0)


def test_sec51_rank_revealing_and_sec52_optimal_error_with_q2():
    """Sec. 5.1/5.2 qualitative claims on the Sec. 5.1 matrix (n = 1000, k = 20,
    l = 2k): the gap after sigma_k is revealed by diag(T) for q = 0 and 2, and
    with q = 2 the rank-k error e_k (eq. 13) equals the SVD optimum."""
    A, _ = sec51_matrix(1000, 20, seed=51)
    s = np.linalg.svd(A, compute_uv=False)
    opt = np.sqrt(np.sum(s[20:] ** 2))
    for q in (0, 2):
        r = corutv(A, 20, 20, q, seed=1)
        d = np.diag(r["T"])
        assert d[19] / d[20] > 5.0
        ek = np.linalg.norm(A - truncate(r["U"], r["T"], r["V"], 20))
        assert ek >= opt * (1 - 1e-9)
        if q == 2:
            assert ek <= opt * (1 + 1e-6)
        else:
            assert ek <= opt * 2.0


def test_power_iterations_improve_accuracy_on_slow_decay():
    """Sec. 3.1: the power method helps when the spectrum decays slowly."""
    A = decaying(400, 300, 300, 0.0, seed=3, kind="poly", alpha=0.3)
    errs = [rel_err(A, **{k: v for k, v in corutv(A, 10, 5, q, seed=2).items() if k in "UTV"})
            for q in (0, 1, 2)]
    assert errs[0] > errs[1] > errs[2]


def test_planted_mistakes_are_caught():
    """A wrong output permutation (V = Q2 P^T, the transposed permutation) or a
    dropped sign normalisation must break the pins above."""
    A = noisy_low_rank(200, 150, 8, 0.0, seed=1)
    r = corutv(A, 8, 4, 0, seed=2)
    inv = np.argsort(r["piv"])
    Vbad = r["Q2"][:, inv]
    if not np.array_equal(inv, r["piv"]):
        assert rel_err(A, r["U"], r["T"], Vbad) > 1e-3
    Tbad = r["T"].copy()
    Tbad[0] *= -1
    assert rel_err(A, r["U"], Tbad, r["V"]) > 1e-3


@pytest.mark.parametrize("q", [0, 1, 2])
def test_single_revisit_core_is_exact_when_the_range_is_captured(q):
    """A of rank r <= l: A = A Q2 Q2^T exactly, so D_approx = Q1^T C1
    (Q2^T Psi)^+ equals D = Q1^T A Q2 (Sec. 3.1): C1 = A Psi = A Q2 Q2^T Psi
    and Q2^T Psi is invertible."""
    rng = np.random.default_rng(40 + q)
    A = rng.standard_normal((300, 12)) @ rng.standard_normal((12, 200))
    a = corutv(A, 15, 5, q, seed=3)
    b = corutv(A, 15, 5, q, seed=3, core="approx")
    nA = np.linalg.norm(A)
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-10 * nA
    assert np.linalg.norm(b["U"] @ b["T"] @ b["V"].T - A) <= 1e-10 * nA


@pytest.mark.parametrize("q", [0, 1])
def test_single_revisit_core_literal_equals_stabilized(q):
    """The stabilized loop's Psi is the literal C2 times an upper triangular
    factor G^-1, and C1 = A Psi carries the same factor, so Q1^T C1 (Q2^T
    Psi)^+ is the same matrix in both modes (App. A.1 with R5's reading)."""
    A = decaying(400, 300, 60, 1e-6, seed=11, kind="exp", tau=8.0)
    a = corutv(A, 10, 5, q, seed=2, mode="literal", core="approx")
    b = corutv(A, 10, 5, q, seed=2, core="approx")
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-8 * np.linalg.norm(A)


@pytest.mark.parametrize("q", [0, 1, 2])
def test_single_revisit_core_equals_the_exact_core(q):
    """Not only for low rank: Q2 spans the range of Z = A^T Q1 (Q2 R_Z = Z),
    so Q1^T A = R_Z^T Q2^T exactly and Q1^T C1 = Q1^T A Psi = R_Z^T (Q2^T Psi).
    Hence D_approx = R_Z^T (Q2^T Psi)(Q2^T Psi)^+ = R_Z^T = D for any A once
    Q2^T Psi has full rank; full-rank noise beyond rank l included."""
    A = decaying(500, 400, 200, 1e-3, seed=5 + q, kind="exp", tau=6.0)
    a = corutv(A, 15, 5, q, seed=9)
    b = corutv(A, 15, 5, q, seed=9, core="approx")
    c = corutv(A, 15, 5, q, seed=9, core="rz")
    nA = np.linalg.norm(A)
    assert np.linalg.norm(b["D"] - a["D"]) <= 1e-10 * nA
    assert np.linalg.norm(b["D"] - c["D"]) <= 1e-10 * nA
    # a planted mistake: the C2 of the final iteration instead of the one
    # that produced C1 (R5) breaks the identity
    if q > 0:
        wrong = a["Q1"].T @ (A @ b["Psi"]) @ np.linalg.pinv(a["Q2"].T @ (A.T @ a["Q1"]))
        assert np.linalg.norm(wrong - a["D"]) > 1e-3 * nA


@pytest.mark.parametrize("m,n,q,tri", [(300, 200, 1, "upper"), (300, 200, 0, "lower"), (150, 260, 2, "auto")])
def test_core_from_rz_gives_the_same_factorization(m, n, q, tri):
    """core="rz" (D = R_Z^T, one product with A fewer) and core="pass" give the
    same rank-l approximation and the same leading pivots: the two cores
    differ only by rounding (Sec. 3.1 eqs. 5-7)."""
    A = decaying(m, n, 80, 1e-6, seed=m + q, kind="exp", tau=6.0)
    a = corutv(A, 15, 5, q, seed=7, tri=tri)
    b = corutv(A, 15, 5, q, seed=7, tri=tri, core="rz")
    nA = np.linalg.norm(A)
    assert np.linalg.norm(a["D"] - b["D"]) <= 1e-13 * nA
    Aa = a["U"] @ a["T"] @ a["V"].T
    Ab = b["U"] @ b["T"] @ b["V"].T
    assert np.linalg.norm(Aa - Ab) <= 1e-12 * nA
    np.testing.assert_array_equal(a["piv"][:10], b["piv"][:10])
    with pytest.raises(ValueError):
        corutv(A, 15, 5, q, seed=7, mode="literal", core="rz")


@pytest.mark.parametrize("m,n,tri", [(150, 260, "auto"), (260, 150, "lower"), (260, 150, "upper")])
def test_truncation_is_a_projection_of_the_approximation(m, n, tri):
    """Rank-r truncation (Sec. 5.2, eq. 12).  Upper T keeps the first r rows
    of T, which is the projection U_r U_r^T A_hat onto the leading left
    vectors; lower T (the transposed problem) keeps the first r columns, the
    projection A_hat V_r V_r^T.  Both follow from U, V orthonormal and T
    triangular, independently of how truncate() is written; a row truncation
    applied to a lower T is a different matrix and must not pass."""
    A = decaying(m, n, 80, 1e-3, seed=m + 2 * n, kind="exp", tau=6.0)
    res = corutv(A, 15, 5, 1, seed=4, tri=tri)
    U, T, V = res["U"], res["T"], res["V"]
    lower = bool(np.all(np.triu(T, 1) == 0))
    assert lower == (tri == "lower" or (tri == "auto" and m < n))
    Ah = U @ T @ V.T
    nA = np.linalg.norm(A)
    for r in (1, 7, 20):
        got = truncate(U, T, V, r, "lower" if lower else "upper")
        if lower:
            want = Ah @ V[:, :r] @ V[:, :r].T
            wrong = U[:, :r] @ T[:r, :] @ V.T
        else:
            want = U[:, :r] @ (U[:, :r].T @ Ah)
            wrong = U @ T[:, :r] @ V[:, :r].T
        assert np.linalg.norm(got - want) <= 1e-13 * nA
        if r < 20:
            assert np.linalg.norm(wrong - want) > 1e-6 * nA
    assert np.linalg.norm(truncate(U, T, V, 20, "lower" if lower else "upper") - Ah) <= 1e-14 * nA


def test_truncation_of_the_wide_problem_is_the_transposed_tall_one():
    """The lower-T truncation of a wide A equals the upper-T truncation of
    the tall A^T, transposed (P13 carried through eq. 12)."""
    A = decaying(120, 300, 40, 1e-4, seed=8)
    a = corutv(A, 10, 5, 1, seed=9)
    b = corutv(A.T.copy(), 10, 5, 1, seed=9, tri="upper")
    for r in (1, 6, 15):
        x = truncate(a["U"], a["T"], a["V"], r, "lower")
        y = truncate(b["U"], b["T"], b["V"], r, "upper")
        assert np.linalg.norm(x - y.T) <= 1e-14 * np.linalg.norm(A)
