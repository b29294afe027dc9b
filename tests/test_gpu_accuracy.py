"""The paper's accuracy claims, on the GPU path (Sec. 5.1, 5.2, Sec. 3.1 and
eq. 3), against mathematical facts rather than the oracle's output: the
Eckart-Young optimum and the randomized range finder's average bound from
the SVD of A, the rank-revealing gap of diag(T), the optimal rank-k error
with power iterations, and the effect of q on a slowly decaying spectrum."""
import numpy as np
import pytest
import torch

from oracle.corutv import truncate
from oracle.dense import jacobi_svd
from workloads import decaying, noisy_low_rank, sec51_matrix

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_04572_amd as cu

    c = cu.Context(workspace_bytes=1 << 30)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _run(ctx, A, k, p, q, seed, prec):
    dt = torch.float64 if prec == "f64" else torch.float32
    U, T, V, piv, info = ctx.decompose(torch.from_numpy(A).to(dt).cuda(), k, p, q, seed, prec=prec)
    return U.cpu().double().numpy(), T.cpu().numpy(), V.cpu().double().numpy()


@pytest.mark.parametrize("q", [0, 2])
def test_sec51_gap_and_sec52_optimal_rank_k_error(ctx, q):
    """Sec. 5.1 matrix (n = 1000, sigma linear from 1 to 1e-9 over k = 20,
    noise 0.1 sigma_k): diag(T) reveals the gap after sigma_20, e_k (eq. 13)
    is never below the SVD optimum, and with q = 2 it equals the optimum."""
    _say("sec51", q)
    A, _ = sec51_matrix(1000, 20, seed=51)
    s = np.linalg.svd(A, compute_uv=False)
    opt = np.sqrt(np.sum(s[20:] ** 2))
    U, T, V = _run(ctx, A, 20, 20, q, 1, "f64")
    d = np.diag(T)
    assert d[19] / d[20] > 5.0
    ek = np.linalg.norm(A - truncate(U, T, V, 20))
    assert ek >= opt * (1 - 1e-9)
    assert ek <= opt * (1 + 1e-6 if q == 2 else 2.0)


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3"])
def test_eckart_young_and_average_case_bound(ctx, prec):
    """eq. 3: e_l >= ||A - A_l||_F for every draw; over 20 draws the mean
    obeys sqrt(1 + k/(p-1)) ||A - A_k||_F (U T V^T = Q1 Q1^T A)."""
    _say("eckart-young", prec)
    A = decaying(200, 150, 150, 0.0, seed=40, kind="poly", alpha=1.0)
    s = jacobi_svd(A)[1]
    k, p = 10, 6
    opt_l = np.sqrt(np.sum(s[k + p:] ** 2))
    opt_k = np.sqrt(np.sum(s[k:] ** 2))
    Ac = A if prec == "f64" else A.astype(np.float32).astype(np.float64)
    errs = []
    for seed in range(20):
        U, T, V = _run(ctx, A, k, p, 0, seed, prec)
        e = np.linalg.norm(Ac - U @ T @ V.T)
        assert e >= opt_l * (1 - 1e-6)
        errs.append(e)
    assert np.mean(errs) <= np.sqrt(1 + k / (p - 1)) * opt_k * 1.1


@pytest.mark.parametrize("prec", ["f32", "bf16x3"])
def test_power_iterations_help_on_slow_decay(ctx, prec):
    """Sec. 3.1: on a slowly decaying spectrum, q = 1 and q = 2 each improve
    the error."""
    _say("power iterations", prec)
    A = decaying(400, 300, 300, 0.0, seed=3, kind="poly", alpha=0.3)
    errs = []
    for q in (0, 1, 2):
        U, T, V = _run(ctx, A, 10, 5, q, 2, prec)
        errs.append(np.linalg.norm(A - U @ T @ V.T) / np.linalg.norm(A))
    assert errs[0] > errs[1] > errs[2]


def test_rank_revealing_gap_and_threshold_rank(ctx):
    """Rank 12 plus 1e-8 noise: T_13,13 / T_12,12 is of the order of the
    noise, and the count of diagonals above a threshold in the gap is 12."""
    _say("rank gap")
    A = noisy_low_rank(300, 250, 12, 1e-8, seed=17)
    U, T, V = _run(ctx, A, 12, 8, 1, 5, "f64")
    d = np.diag(T)
    assert d[12] / d[11] < 1e-6
    delta = np.sqrt(d[11] * d[12])
    assert int(np.sum(d > delta)) == 12


@pytest.mark.slow
def test_sec5_studies_against_oracle(ctx):
    """The Sec. 5.1 and 5.2 studies on the GPU path (F64), each draw compared
    with the oracle run on the same seed.  Matrix of Sec. 5.1 (n = 1000,
    rank k = 20, sigma_i linear from 1 to 1e-9, noise 0.1 sigma_k E with
    ||E||_2 = 1); 20 trials (test-matrix seeds 1..20) for q = 0 and q = 2.

    Fig. 1: mean over the trials of diag(T)_i / sigma_i(A), l = 2k = 40.
    The leading 19 entries (sigma_i >= 0.05) must agree with the oracle's to
    1e-10 relative; the trailing ones (sigma_20 = 1e-9 and the 1e-10 noise
    level, where Householder rounding of order u ||A|| already perturbs the
    sketch's trailing directions, and pivots among noise-level columns are
    not unique) are reported and bounded loosely (1e-3 relative).
    Fig. 2: mean e_k = ||A - U(:, 1:k) T(1:k, :) V^T||_F (eq. 13, rank
    k = 20) against l; each draw's e_k within 1e-13 (about 40 u ||A||_F)
    of the oracle's.  Both sides must show what the paper reports: e_k never
    below the SVD optimum, and with q = 2 equal to it (1e-6 relative; 1e-5
    for l = k, i.e. without oversampling)."""
    from oracle.corutv import corutv

    A, _ = sec51_matrix(1000, 20, seed=51)
    s = np.linalg.svd(A, compute_uv=False)
    opt = float(np.sqrt(np.sum(s[20:] ** 2)))
    k, trials = 20, 20
    ells = (20, 24, 30, 40, 50, 60, 80)
    Ad = torch.from_numpy(A).cuda()
    print("\nSec. 5.1 / 5.2 studies, n = 1000, k = 20, %d trials; SVD optimum e_k = %.6e" % (trials, opt))
    for q in (0, 2):
        _say("sec5 studies q=%d" % q)
        ek_g = {ell: [] for ell in ells}
        ek_o = {ell: [] for ell in ells}
        dg_g, dg_o = [], []
        for ell in ells:
            for seed in range(1, trials + 1):
                U, T, V, piv, info = ctx.decompose(Ad, k, ell - k, q, seed, prec="f64")
                Ug, Tg, Vg = U.cpu().numpy(), T.cpu().numpy(), V.cpu().numpy()
                r = corutv(A, k, ell - k, q, seed=seed)
                eg = np.linalg.norm(A - truncate(Ug, Tg, Vg, k))
                eo = np.linalg.norm(A - truncate(r["U"], r["T"], r["V"], k))
                assert abs(eg - eo) <= 1e-13, (q, ell, seed, eg, eo)
                assert eg >= opt * (1 - 1e-9) and eo >= opt * (1 - 1e-9)
                ek_g[ell].append(eg)
                ek_o[ell].append(eo)
                if ell == 2 * k:
                    dg_g.append(np.diag(Tg))
                    dg_o.append(np.diag(r["T"]))
        rg = np.mean(dg_g, axis=0) / s[:2 * k]
        ro = np.mean(dg_o, axis=0) / s[:2 * k]
        lead = np.max(np.abs(rg[:19] - ro[:19]))
        tail = np.max(np.abs(rg[19:] - ro[19:]) / np.abs(ro[19:]))
        print("q=%d Fig. 1: mean diag(T)_i / sigma_i, GPU (oracle):" % q)
        for i in (0, 4, 9, 14, 18, 19, 20, 29, 39):
            print("   i=%2d  sigma %.4e  %.10f (%.10f)" % (i + 1, s[i], rg[i], ro[i]))
        print("   max |GPU - oracle|: leading 19 %.2e, trailing (relative) %.2e" % (lead, tail))
        assert lead <= 1e-10
        assert tail <= 1e-3
        print("q=%d Fig. 2: mean e_k / SVD optimum against l, GPU (oracle):" % q)
        for ell in ells:
            mg, mo = np.mean(ek_g[ell]), np.mean(ek_o[ell])
            print("   l=%2d  %.10f (%.10f)" % (ell, mg / opt, mo / opt))
            if q == 2:  # no oversampling (l = k) leaves 1.1e-6 on both sides
                bound = 1e-6 if ell > k else 1e-5
                assert mg <= opt * (1 + bound) and mo <= opt * (1 + bound)
