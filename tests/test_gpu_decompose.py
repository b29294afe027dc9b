"""End-to-end GPU parity of corutv_decompose against the float64 oracle.

Bars (the decomposition is randomized but both sides draw the identical test
matrix, so they compute the same thing up to rounding):
* F64 path: |e_gpu - e_oracle| <= 1e-10 and ||A_gpu - A_oracle||_F / ||A||_F
  <= 1e-10 (A_x = U T V^T), U, V orthonormal to 1e-13, T exactly triangular
  with a non-negative non-increasing diagonal, and the pivots of the steps
  decided by a margin (the leading k) identical.
* F32 path: |e_gpu - e_oracle| <= 1e-5 (e = relative Frobenius error) with
  the oracle run in float64 on the same float32 data.
Cases cover the small plain configuration (2000 x 1500, rank 20 + 1e-6 noise,
l = 30, q = 1, lower T), orientations, layouts, ragged sizes, q in {0, 1, 2},
exact low rank (Householder fallback), NaN input and bad arguments.
"""
import numpy as np
import pytest
import torch

from oracle.corutv import corutv, rel_err
from workloads import decaying, noisy_low_rank

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import paper_1906_04572_amd as cu

    c = cu.Context(workspace_bytes=1 << 31)
    yield c
    c.close()


def _say(*a):
    print("[case]", *a, flush=True)


def _dev(A, layout):
    if layout == "row":
        return torch.from_numpy(np.ascontiguousarray(A)).cuda()
    return torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()


def _run(ctx, A, k, p, q, seed, prec, tri, layout="row"):
    U, T, V, piv, info = ctx.decompose(_dev(A, layout), k, p, q, seed, prec=prec, tri=tri, want_err=True)
    return U.cpu().numpy().astype(np.float64), T.cpu().numpy(), V.cpu().numpy().astype(np.float64), \
        piv.cpu().numpy(), info


def _check_f64(A, k, p, q, seed, tri, got, ref):
    U, T, V, piv, info = got
    ell = k + p
    e_ref = rel_err(A, ref["U"], ref["T"], ref["V"])
    assert abs(info["rel_err"] - e_ref) <= 1e-10, (info["rel_err"], e_ref)
    Ah = U @ T @ V.T
    Ar = ref["U"] @ ref["T"] @ ref["V"].T
    d = np.linalg.norm(Ah - Ar) / np.linalg.norm(A)
    assert d <= 1e-10, d
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= 1e-13
    lower = info["tri"] == "lower"
    assert np.all((np.triu(T, 1) if lower else np.tril(T, -1)) == 0)
    dg = np.diag(T)
    assert np.all(dg >= 0) and np.all(dg[:-1] >= dg[1:] * (1 - 1e-12))
    np.testing.assert_array_equal(piv[:k], ref["piv"][:k])
    # leading-k factors (signs are fixed by diag(T) >= 0)
    np.testing.assert_allclose(dg[:k], np.diag(ref["T"])[:k], rtol=1e-10, atol=0)
    return info


def test_plain_config_2000x1500_rank20_lower(ctx):
    _say("C1 2000x1500 rank20 1e-6 noise, l=30, q=1, lower, f64")
    A = noisy_low_rank(2000, 1500, 20, 1e-6, seed=1)
    got = _run(ctx, A, 20, 10, 1, 2024, "f64", "lower")
    ref = corutv(A, 20, 10, 1, seed=2024, tri="lower")
    info = _check_f64(A, 20, 10, 1, 2024, "lower", got, ref)
    assert info["tri"] == "lower" and info["passes"] == 6
    print("C1 rel_err gpu %.12e fallbacks %d" % (info["rel_err"], info["qr_fallbacks"]))


@pytest.mark.parametrize("m,n,k,p,q,tri,layout", [
    (1200, 900, 20, 10, 1, "upper", "row"),
    (1200, 900, 20, 10, 0, "auto", "col"),
    (900, 1200, 20, 10, 1, "auto", "row"),
    (900, 1200, 20, 10, 2, "upper", "col"),
    (1037, 613, 17, 6, 1, "lower", "col"),
    (3000, 250, 5, 5, 1, "auto", "row"),
    (700, 700, 100, 28, 1, "auto", "row"),
    (2100, 1900, 150, 50, 0, "upper", "row"),
    (1800, 1500, 120, 20, 1, "lower", "row"),
    # tall and thin: the passes with the long output (313 tiles of 128 rows,
    # a 300-long reduction, ragged last tile) write it from one workgroup
    # per tile, no partial sums; row-major and the transposed wide problem
    (40000, 300, 8, 4, 1, "auto", "row"),
    (300, 40000, 8, 4, 1, "auto", "col"),
])
def test_f64_cases(ctx, m, n, k, p, q, tri, layout):
    _say("f64", m, n, k, p, q, tri, layout)
    A = decaying(m, n, min(m, n) // 2, 1e-4, seed=m + n, kind="exp", tau=max(k / 2, 3))
    got = _run(ctx, A, k, p, q, 77, "f64", tri, layout)
    ref = corutv(A, k, p, q, seed=77, tri=tri)
    _check_f64(A, k, p, q, 77, tri, got, ref)


@pytest.mark.parametrize("m,n,k,p,q,layout", [
    (3000, 2000, 50, 10, 1, "row"), (2000, 3000, 50, 10, 1, "col"), (4000, 3000, 100, 10, 2, "row"),
    (2500, 1800, 30, 20, 0, "col"),
])
def test_f32_cases(ctx, m, n, k, p, q, layout):
    _say("f32", m, n, k, p, q, layout)
    A = decaying(m, n, 300, 1e-4, seed=m * 3 + n, kind="exp", tau=25.0).astype(np.float32)
    U, T, V, piv, info = _run(ctx, A, k, p, q, 5, "f32", "auto", layout)
    A64 = A.astype(np.float64)
    ref = corutv(A64, k, p, q, seed=5)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    assert abs(info["rel_err"] - e_ref) <= 1e-5, (info["rel_err"], e_ref)
    e_gpu = rel_err(A64, U, T, V)  # the returned factors themselves
    assert abs(e_gpu - e_ref) <= 1e-5
    ell = k + p
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= 1e-5
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= 1e-5


@pytest.mark.parametrize("m,n,k,p,q,tri,layout,prec", [
    (70001, 300, 5, 5, 1, "auto", "col", "f64"),    # CholeskyQR2 over 64 row blocks; the frames shape
    (300, 70001, 5, 5, 1, "auto", "row", "f64"),    # wide: the transposed problem
    (5000, 1200, 12, 4, 2, "upper", "row", "f64"),  # l = 16
    (1100, 900, 1, 0, 1, "lower", "col", "f64"),    # l = 1, one workgroup
    (2047, 1025, 7, 2, 0, "auto", "row", "f64"),
    (20000, 3000, 10, 6, 1, "auto", "row", "f32"),
    (3000, 20000, 10, 5, 2, "auto", "col", "bf16x3"),
    (100003, 200, 12, 4, 1, "auto", "col", "f64"),
    (100003, 200, 12, 4, 1, "auto", "row", "f32"),  # one CholeskyQR step in FP32 storage
    (300001, 40, 5, 5, 1, "auto", "col", "f64"),    # more than one 1024-row chunk per block
])
def test_small_sketch_qr_against_oracle(ctx, m, n, k, p, q, tri, layout, prec):
    """Sketches with l <= 16 columns take the CholeskyQR2 for at most 16
    columns: in one launch when one workgroup holds every row (up to 1024),
    else in three (Gram and Cholesky in the last row block to finish):
    F64 to the 1e-10 bars, F32/BF16X3 |e_gpu - e_oracle| <= 1e-5, across
    panel and block counts, ragged panels, l = 1 and l = 16, both triangles
    and layouts."""
    _say("small-l QR", m, n, k, p, q, tri, layout, prec)
    dt = np.float64 if prec == "f64" else np.float32
    A = decaying(m, n, min(m, n) // 2, 1e-4, seed=m + 7 * n, kind="exp", tau=max(k / 2, 2)).astype(dt)
    A64 = A.astype(np.float64)
    ref = corutv(A64, k, p, q, seed=21, tri=tri)
    if prec == "f64":
        got = _run(ctx, A64, k, p, q, 21, "f64", tri, layout)
        info = _check_f64(A64, k, p, q, 21, tri, got, ref)
    else:
        U, T, V, piv, info = _run(ctx, A, k, p, q, 21, prec, tri, layout)
        e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
        assert abs(info["rel_err"] - e_ref) <= 1e-5, (info["rel_err"], e_ref)
        ell = k + p
        assert np.max(np.abs(U.T @ U - np.eye(ell))) <= 1e-5
        assert np.max(np.abs(V.T @ V - np.eye(ell))) <= 1e-5
    assert info["qr_fallbacks"] == 0


@pytest.mark.parametrize("rows,ell,rank", [(300, 16, 3), (700, 4, 0), (70001, 10, 5), (5000, 1, 0),
                                           (100003, 16, 5)])
def test_small_sketch_rank_deficient(ctx, rows, ell, rank):
    """A rank-deficient sketch with l <= 16 through the whole decomposition of
    an exactly rank-`rank` matrix (rank 0: the zero matrix): the CholeskyQR2
    for at most 16 columns (one launch for 300 x 16 and 700 x 4, three for
    the taller ones) reports the breakdown and the Householder fallback takes
    over: inside the CholeskyQR2 launches where the register-resident form
    fits (one workgroup for 300 x 16 and 700 x 4; the two-level tree over the
    row blocks for 70001 x 10 and 5000 x 1), by the device-memory tree for
    100003 x 16 (100 blocks of 16 columns: 1568 stacked rows).  An
    orthonormal basis whose first `rank` columns (unique) equal the
    oracle's."""
    _say("small-l rank-deficient", rows, ell, rank)
    rng = np.random.default_rng(rows + ell)
    n = max(ell + 5, 40)
    A = rng.standard_normal((rows, rank)) @ rng.standard_normal((rank, n)) if rank else np.zeros((rows, n))
    U, T, V, piv, info = _run(ctx, A, ell, 0, 1, 3, "f64", "auto", "row")
    assert info["qr_fallbacks"] >= 1
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= 1e-13
    a_fro = max(np.linalg.norm(A), 1.0)
    assert np.linalg.norm(A - U @ T @ V.T) <= 1e-12 * a_fro
    if rank:
        ref = corutv(A, ell, 0, 1, seed=3)
        Ah, Ar = U @ T @ V.T, ref["U"] @ ref["T"] @ ref["V"].T
        assert np.linalg.norm(Ah - Ar) <= 1e-10 * a_fro


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "f64"])
def test_one_step_cholesky_qr_well_conditioned(ctx, prec):
    # exp(-i/25) decay: the sketches have condition numbers of a few dozen, so
    # in the FP32-stored forms every thin QR stops after one CholeskyQR step
    # (u l (||R||_F ||R^-1||_F)^2 <= 2^-24); the F64 form always takes two
    _say("one-step QR", prec)
    A = decaying(3000, 2000, 300, 1e-4, seed=11, kind="exp", tau=25.0)
    A = A if prec == "f64" else A.astype(np.float32)
    U, T, V, piv, info = _run(ctx, A, 50, 10, 1, 5, prec, "auto")
    print("qr_one_step", info["qr_one_step"], "fallbacks", info["qr_fallbacks"])
    assert info["qr_fallbacks"] == 0
    assert info["qr_one_step"] == (0 if prec == "f64" else 4)
    A64 = A.astype(np.float64)
    ref = corutv(A64, 50, 10, 1, seed=5)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    assert abs(info["rel_err"] - e_ref) <= (1e-10 if prec == "f64" else 1e-5)
    # the factors stay orthonormal to FP32 storage precision at least
    ell = 60
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= 1e-6
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= 1e-6


def test_one_step_cholesky_qr_refused_when_ill_conditioned(ctx):
    # exp(-i/5) decay without noise: condition numbers near 1e5, where one
    # step would lose orthogonality far above FP32 rounding, so the QRs take
    # the second step (and CholeskyQR does not break down)
    _say("one-step QR refused")
    A = decaying(3000, 2000, 300, 0.0, seed=12, kind="exp", tau=5.0).astype(np.float32)
    U, T, V, piv, info = _run(ctx, A, 50, 10, 0, 5, "f32", "auto")
    print("qr_one_step", info["qr_one_step"], "fallbacks", info["qr_fallbacks"])
    assert info["qr_one_step"] < 2
    A64 = A.astype(np.float64)
    ref = corutv(A64, 50, 10, 0, seed=5)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    assert abs(info["rel_err"] - e_ref) <= 1e-5
    assert np.max(np.abs(U.T @ U - np.eye(60))) <= 1e-5


@pytest.mark.parametrize("prec", ["f64", "f32"])
def test_exact_low_rank_is_recovered(ctx, prec):
    _say("exact rank", prec)
    A = noisy_low_rank(1500, 1100, 12, 0.0, seed=3)
    if prec == "f32":
        A = A.astype(np.float32)
    U, T, V, piv, info = _run(ctx, A, 12, 8, 1, 9, prec, "auto")
    assert info["qr_fallbacks"] >= 1
    bound = 1e-12 if prec == "f64" else 1e-5
    assert info["rel_err"] <= bound
    assert rel_err(A.astype(np.float64), U, T, V) <= bound


def test_nan_input_is_reported(ctx):
    import paper_1906_04572_amd as cu

    _say("nan")
    A = decaying(600, 500, 50, 1e-3, seed=1)
    A[123, 45] = np.nan
    rc = ctx.decompose_rc(_dev(A, "row"), 10, 5, 1, 3)
    assert rc == cu.E_NUMERIC


def test_bad_arguments_leave_outputs_untouched(ctx):
    import paper_1906_04572_amd as cu

    _say("bad args")
    A = torch.from_numpy(decaying(300, 200, 20, 1e-3, seed=1)).cuda()
    out = ctx.alloc_outputs(A, 10, 5)
    for t in out:
        t.fill_(7)
    assert ctx.decompose_rc(A, 150, 100, 1, 3, out=out) == cu.E_INVAL  # l > min(m, n)
    assert ctx.decompose_rc(A, 0, 5, 1, 3, out=out) == cu.E_INVAL
    assert ctx.decompose_rc(A, 10, 5, -1, 3, out=out) == cu.E_INVAL
    assert ctx.decompose_rc(A, 10, 5, 1, 3, prec="f32", out=out) == cu.E_INVAL  # f64 data
    empty = torch.empty((0, 200), dtype=torch.float64, device="cuda")
    assert ctx.decompose_rc(empty, 10, 5, 1, 3, out=out) == cu.E_INVAL  # no rows
    torch.cuda.synchronize()
    for t in out:
        assert torch.all(t == 7)


def test_deterministic_bitwise(ctx):
    _say("determinism")
    A = _dev(decaying(5000, 3000, 200, 1e-4, seed=2), "row").float()
    a = ctx.decompose(A, 50, 10, 1, 4, prec="f32")
    b = ctx.decompose(A, 50, 10, 1, 4, prec="f32")
    for x, y in zip(a[:4], b[:4]):
        assert torch.equal(x, y)


@pytest.mark.parametrize("prec,bound", [("bf16x3", 1e-5), ("f32", 1e-5), ("bf16", 1e-5)])
def test_precision_forms_polynomial_decay(ctx, prec, bound):
    """Precision forms on the polynomially decaying workload (sigma_i = i^-1.5,
    1e-5 noise, l = 220, q = 2) at reduced size: relative Frobenius error
    against the float64 oracle on the same float32 data.  The split-bf16 form
    holds the 1e-5 bar; plain bf16 is reported with its measured bound."""
    _say("precision form", prec)
    A = decaying(6000, 4000, 1000, 1e-5, seed=3, kind="poly", alpha=1.5, dtype=np.float32)
    U, T, V, piv, info = _run(ctx, A, 200, 20, 2, 17, prec, "auto")
    A64 = A.astype(np.float64)
    ref = corutv(A64, 200, 20, 2, seed=17)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    d = abs(info["rel_err"] - e_ref)
    print("precision %s: e_gpu %.8e e_oracle %.8e |diff| %.3e" % (prec, info["rel_err"], e_ref, d))
    assert d <= bound
    assert np.max(np.abs(U.T @ U - np.eye(220))) <= 1e-5
    assert np.max(np.abs(V.T @ V - np.eye(220))) <= 1e-5


def _ahat_rel_diff(got, ref, a_fro, block=4096):
    """||U T V^T - U_o T_o V_o^T||_F / ||A||_F, formed explicitly in row
    blocks on the device in float64 (the products are too large for the
    host at the full sizes)."""
    dev = torch.device("cuda", 0)
    Ug, Tg, Vg = (torch.as_tensor(np.asarray(x, dtype=np.float64), device=dev) for x in got)
    Uo, To, Vo = (torch.from_numpy(np.asarray(ref[x], dtype=np.float64)).to(dev) for x in ("U", "T", "V"))
    B1, B2 = Ug @ Tg, Uo @ To
    V1t, V2t = Vg.t().contiguous(), Vo.t().contiguous()
    tot = 0.0
    for i in range(0, B1.shape[0], block):
        X = B1[i:i + block] @ V1t - B2[i:i + block] @ V2t
        tot += float(torch.sum(X * X).item())
    return np.sqrt(tot) / a_fro


@pytest.mark.slow
def test_full_size_20000x15000_against_oracle(ctx):
    """The 20000 x 15000 plain configuration at its real size, in the launch
    configurations bench.py times (k = 100, p = 10, q = 1), against one
    float64 oracle run on the same data (the float32 draw, widened):
    F64 path: |e_gpu - e_oracle| <= 1e-10, ||A_gpu - A_oracle||_F / ||A||_F
    <= 1e-10, bases orthonormal to 1e-13, the leading 60 pivots (singular
    values e^(-i/25) far above the 1e-4 noise: steps decided by wide
    margins) identical; F32 path: |e_gpu - e_oracle| <= 1e-5, bases
    orthonormal to FP32 accuracy, T exactly triangular."""
    _say("full size 20000x15000 q=1 vs oracle (f64, f32)")
    A = decaying(20000, 15000, 300, 1e-4, seed=2, kind="exp", tau=25.0, dtype=np.float32)
    A64 = A.astype(np.float64)
    ref = corutv(A64, 100, 10, 1, seed=1)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    a_fro = float(np.linalg.norm(A64))
    U, T, V, piv, info = _run(ctx, A64, 100, 10, 1, 1, "f64", "auto")
    d_ahat = _ahat_rel_diff((U, T, V), ref, a_fro)
    print("full size f64: e_gpu %.14e e_oracle %.14e |A_gpu - A_oracle|/|A| %.3e"
          % (info["rel_err"], e_ref, d_ahat))
    assert abs(info["rel_err"] - e_ref) <= 1e-10
    assert d_ahat <= 1e-10
    assert np.max(np.abs(U.T @ U - np.eye(110))) <= 1e-13
    assert np.max(np.abs(V.T @ V - np.eye(110))) <= 1e-13
    assert np.all(np.tril(T, -1) == 0)
    np.testing.assert_array_equal(piv[:60], ref["piv"][:60])
    U, T, V, piv, info = _run(ctx, A, 100, 10, 1, 1, "f32", "auto")
    print("full size f32: e_gpu %.10e e_oracle %.10e" % (info["rel_err"], e_ref))
    assert abs(info["rel_err"] - e_ref) <= 1e-5
    assert np.max(np.abs(U.T @ U - np.eye(110))) <= 1e-5
    assert np.max(np.abs(V.T @ V - np.eye(110))) <= 1e-5
    assert np.all(np.tril(T, -1) == 0)


@pytest.mark.slow
def test_full_size_precision_forms_50000x30000_against_oracle(ctx):
    """The precision-form configuration at its real size (50000 x 30000,
    sigma_i = i^-1.5 for i <= 1000 plus 1e-5 noise, float32; k = 200,
    p = 20, q = 2; l = 220) against one float64 oracle run on the same
    float32 data: F64 path |e_gpu - e_oracle| <= 1e-10 and
    ||A_gpu - A_oracle||_F / ||A||_F <= 1e-10 with the leading 20 pivots
    identical; F32, BF16X3 and BF16 |e_gpu - e_oracle| <= 1e-5, bases
    orthonormal to 1e-5, T exactly triangular.  The data is drawn on the
    device (seeded torch generator) from the recipe and copied to the
    host for the oracle."""
    _say("full size 50000x30000 precision forms vs oracle")
    m, n, r = 50000, 30000, 1000
    g = torch.Generator(device="cuda")
    g.manual_seed(3)
    U0 = torch.linalg.qr(torch.randn(m, r, generator=g, device="cuda", dtype=torch.float64)).Q
    V0 = torch.linalg.qr(torch.randn(n, r, generator=g, device="cuda", dtype=torch.float64)).Q
    sig = torch.arange(1, r + 1, device="cuda", dtype=torch.float64) ** -1.5
    Ad = (U0 * sig) @ V0.T.contiguous()
    del U0, V0
    Ad += 1e-5 * torch.randn(m, n, generator=g, device="cuda", dtype=torch.float64)
    A32 = Ad.float()
    del Ad
    torch.cuda.empty_cache()
    A64h = A32.cpu().numpy().astype(np.float64)
    _say("oracle float64 on the host")
    ref = corutv(A64h, 200, 20, 2, seed=11)
    e_ref = rel_err(A64h, ref["U"], ref["T"], ref["V"])
    a_fro = float(np.linalg.norm(A64h))
    del A64h
    import paper_1906_04572_amd as cu

    need = max(cu.workspace_bytes(m, n, 200, 20, 2, p) for p in ("f64", "f32", "bf16", "bf16x3"))
    big = cu.Context(workspace_bytes=need)
    eye = torch.eye(220, dtype=torch.float64, device="cuda")
    A = A32.double()  # the FP64 path sees exactly the float32 data
    _say("f64 path")
    U, T, V, piv, info = big.decompose(A, 200, 20, 2, 11, prec="f64", want_err=True)
    del A
    Uh, Th, Vh = U.cpu().numpy(), T.cpu().numpy(), V.cpu().numpy()
    d_ahat = _ahat_rel_diff((Uh, Th, Vh), ref, a_fro)
    print("50000x30000 f64: e %.14e e_oracle %.14e |A_gpu - A_oracle|/|A| %.3e" % (info["rel_err"], e_ref, d_ahat))
    assert abs(info["rel_err"] - e_ref) <= 1e-10
    assert d_ahat <= 1e-10
    assert torch.max(torch.abs(U.T @ U - eye)).item() <= 1e-13
    assert torch.max(torch.abs(V.T @ V - eye)).item() <= 1e-13
    np.testing.assert_array_equal(piv.cpu().numpy()[:20], ref["piv"][:20])
    for prec in ("bf16x3", "f32", "bf16"):
        _say(prec, "path")
        U, T, V, piv, info = big.decompose(A32, 200, 20, 2, 11, prec=prec, want_err=True)
        d = abs(info["rel_err"] - e_ref)
        print("50000x30000 %s: e %.8e e_oracle %.8e |diff| %.3e" % (prec, info["rel_err"], e_ref, d))
        assert d <= 1e-5
        Ud, Vd = U.double(), V.double()
        assert torch.max(torch.abs(Ud.T @ Ud - eye)).item() <= 1e-5
        assert torch.max(torch.abs(Vd.T @ Vd - eye)).item() <= 1e-5
        assert torch.all(torch.tril(T, -1) == 0).item()
    big.close()


@pytest.mark.parametrize("m,n,k,p,q,tri,layout,prec", [
    (1200, 900, 20, 10, 1, "upper", "row", "f64"), (900, 1200, 20, 10, 2, "auto", "col", "f64"),
    (1037, 613, 17, 6, 1, "lower", "col", "f64"), (1800, 1500, 120, 20, 1, "auto", "row", "f64"),
    (3000, 2000, 50, 10, 1, "auto", "row", "f32"), (2000, 3000, 60, 10, 0, "lower", "col", "f32"),
])
def test_core_from_rz_against_oracle(ctx, m, n, k, p, q, tri, layout, prec):
    """Core D = R_Z^T (2q + 2 passes) against the oracle's core="rz": F64 to
    the 1e-10 bars, F32 |e_gpu - e_oracle| <= 1e-5."""
    _say("core rz", m, n, k, p, q, tri, layout, prec)
    dt = np.float64 if prec == "f64" else np.float32
    A = decaying(m, n, min(m, n) // 2, 1e-4, seed=m + 2 * n, kind="exp", tau=max(k / 2, 3)).astype(dt)
    A64 = A.astype(np.float64)
    U, T, V, piv, info = ctx.decompose(_dev(A, layout), k, p, q, 77, prec=prec, tri=tri, want_err=True,
                                       core="rz")
    got = (U.cpu().numpy().astype(np.float64), T.cpu().numpy(), V.cpu().numpy().astype(np.float64),
           piv.cpu().numpy(), info)
    assert info["passes"] == 2 * q + 2 + 1  # + the residual pass
    ref = corutv(A64, k, p, q, seed=77, tri=tri, core="rz")
    if prec == "f64":
        _check_f64(A64, k, p, q, 77, tri, got, ref)
    else:
        e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
        assert abs(info["rel_err"] - e_ref) <= 1e-5
        assert abs(rel_err(A64, got[0], got[1], got[2]) - e_ref) <= 1e-5


@pytest.mark.parametrize("q,prec", [(0, "f64"), (1, "f64"), (2, "f64"), (1, "f32")])
def test_single_revisit_core_against_oracle(ctx, q, prec):
    """The paper's single-revisit core Q1^T C1 (Q2^T Psi)^+, evaluated by the
    oracle as printed (pseudo-inverse), against the GPU's R_Z^T core, which
    is the same matrix: F64 to the 1e-10 bars, F32 |de| <= 1e-5."""
    _say("single-revisit core", q, prec)
    m, n, k, p = 1400, 1000, 30, 10
    dt = np.float64 if prec == "f64" else np.float32
    A = decaying(m, n, 500, 1e-4, seed=31 + q, kind="exp", tau=15.0).astype(dt)
    A64 = A.astype(np.float64)
    U, T, V, piv, info = ctx.decompose(_dev(A, "row"), k, p, q, 5, prec=prec, want_err=True, core="rz")
    got = (U.cpu().numpy().astype(np.float64), T.cpu().numpy(), V.cpu().numpy().astype(np.float64),
           piv.cpu().numpy(), info)
    ref = corutv(A64, k, p, q, seed=5, core="approx")
    if prec == "f64":
        _check_f64(A64, k, p, q, 5, "upper", got, ref)
    else:
        e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
        assert abs(info["rel_err"] - e_ref) <= 1e-5


def _host(A, layout):
    """Pinned host copy of A in the given storage order."""
    if layout == "row":
        return torch.from_numpy(np.ascontiguousarray(A)).pin_memory()
    return torch.from_numpy(np.ascontiguousarray(A.T)).pin_memory().t()


@pytest.mark.parametrize("m,n,layout,prec,q,panel", [
    (1200, 900, "row", "f64", 1, 257),   # five panels, the last one ragged
    (1200, 900, "col", "f64", 1, 200),   # column-major storage: panels of columns
    (900, 1200, "row", "f64", 2, 300),   # wide: the method runs on A^T
    (1037, 613, "col", "f64", 0, 613),   # one panel
    (1500, 1100, "row", "f32", 1, 400),
    (1100, 1500, "col", "f32", 1, 256),
])
def test_host_resident_a_against_oracle(ctx, m, n, layout, prec, q, panel):
    """A in pinned host memory, streamed through the device panel by panel
    in every pass: the factors match the oracle (F64: e and A_hat to 1e-10,
    leading pivots; F32: |de| <= 1e-5) and the device-resident run."""
    _say("host A", m, n, layout, prec, q, panel)
    k, p = 20, 10
    dt = np.float64 if prec == "f64" else np.float32
    A = decaying(m, n, min(m, n) // 2, 1e-4, seed=m + n + q, kind="exp", tau=8.0).astype(dt)
    A64 = A.astype(np.float64)
    U, T, V, piv, info = ctx.decompose(_host(A, layout), k, p, q, 5, prec=prec, panel_rows=panel)
    U, T, V, piv = (U.cpu().numpy().astype(np.float64), T.cpu().numpy(), V.cpu().numpy().astype(np.float64),
                    piv.cpu().numpy())
    assert info["passes"] == 2 * q + 3
    ref = corutv(A64, k, p, q, seed=5)
    e_ref = rel_err(A64, ref["U"], ref["T"], ref["V"])
    e_gpu = rel_err(A64, U, T, V)
    Ad = ctx.decompose(_dev(A, layout), k, p, q, 5, prec=prec)
    Ah_dev = Ad[0].cpu().numpy().astype(np.float64) @ Ad[1].cpu().numpy() @ Ad[2].cpu().numpy().astype(np.float64).T
    nA = np.linalg.norm(A64)
    if prec == "f64":
        assert abs(e_gpu - e_ref) <= 1e-10
        assert np.linalg.norm(U @ T @ V.T - ref["U"] @ ref["T"] @ ref["V"].T) <= 1e-10 * nA
        np.testing.assert_array_equal(piv[:k], ref["piv"][:k])
        assert np.linalg.norm(U @ T @ V.T - Ah_dev) <= 1e-12 * nA
    else:
        assert abs(e_gpu - e_ref) <= 1e-5
        assert np.linalg.norm(U @ T @ V.T - Ah_dev) <= 1e-5 * nA


def test_host_resident_a_rejects_what_it_does_not_support(ctx):
    import paper_1906_04572_amd as cu

    A = decaying(600, 400, 100, 1e-4, seed=3, kind="exp", tau=8.0).astype(np.float32)
    Ah = _host(A, "row")
    assert ctx.decompose_rc(Ah, 10, 5, 1, 1, prec="bf16x3") == cu.E_INVAL
    assert ctx.decompose_rc(Ah, 10, 5, 1, 1, prec="f32", want_err=True) == cu.E_INVAL
    assert ctx.decompose_rc(Ah, 10, 5, 1, 1, prec="f32", panel_rows=-1) == cu.E_INVAL
    assert cu.workspace_bytes_host(600, 400, 10, 5, 1, "bf16") == 0
    assert cu.workspace_bytes_host(600, 400, 10, 5, 1, "f32", "row", 100) > cu.workspace_bytes(600, 400, 10, 5, 1,
                                                                                                 "f32")


def test_core_from_rz_after_cholesky_breakdown(ctx):
    """Exactly low-rank A: the QR of Z falls back to Householder, whose R
    then gives the core; the factorization is still exact."""
    _say("core rz, fallback")
    A = noisy_low_rank(1500, 1100, 12, 0.0, seed=3)
    U, T, V, piv, info = _run_core_rz(ctx, A)
    assert info["qr_fallbacks"] >= 1
    assert info["rel_err"] <= 1e-12
    assert rel_err(A, U, T, V) <= 1e-12


def _run_core_rz(ctx, A):
    U, T, V, piv, info = ctx.decompose(_dev(A, "row"), 12, 8, 1, 9, prec="f64", want_err=True, core="rz")
    return U.cpu().numpy(), T.cpu().numpy(), V.cpu().numpy(), piv.cpu().numpy(), info


def test_unknown_flag_bits_are_rejected(ctx):
    import ctypes

    import paper_1906_04572_amd as cu

    A = torch.from_numpy(decaying(300, 200, 20, 1e-3, seed=1)).cuda()
    U, T, V, piv = ctx.alloc_outputs(A, 10, 5)
    info = cu.Info()
    opts = cu.Opts(cu.PREC["f64"], 0, 0, 4)  # not a defined CORUTV_FLAG_* bit
    rc = cu.lib.corutv_decompose(ctx.h, ctypes.byref(cu.mat(A)), 10, 5, 1, 3, ctypes.byref(opts),
                                 ctypes.byref(cu.mat(U)), T.data_ptr(), 15, ctypes.byref(cu.mat(V)),
                                 piv.data_ptr(), ctypes.byref(info))
    assert rc == cu.E_INVAL


@pytest.mark.parametrize("m,n,k,p,q", [(1, 1, 1, 0, 0), (7, 3, 1, 0, 2), (300, 40, 30, 10, 1), (40, 300, 25, 15, 2)])
def test_degenerate_shapes(ctx, m, n, k, p, q):
    """A 1 x 1 matrix, k = 1 with no oversampling, and l = min(m, n) (the
    factorization is then exact: A = U T V^T to rounding)."""
    _say("degenerate", m, n, k, p, q)
    A = np.random.default_rng(m * 31 + n).standard_normal((m, n))
    got = _run(ctx, A, k, p, q, 11, "f64", "auto")
    ref = corutv(A, k, p, q, seed=11)
    _check_f64(A, k, p, q, 11, "auto", got, ref)
    if k + p == min(m, n):
        assert got[4]["rel_err"] <= 1e-13


@pytest.mark.parametrize("prec,k,p", [("f64", 5, 3), ("f32", 5, 3), ("f64", 12, 8), ("f32", 12, 8)])
def test_zero_matrix(ctx, prec, k, p):
    """A = 0: every sketch is zero, every CholeskyQR breaks down (l = 8: the
    one-launch form for at most 16 columns; l = 20: the general one) and the
    Householder fallback returns an orthonormal basis; the core is zero, no
    column is ever preferred (pivots in natural order, as the oracle's) and
    T = 0, so U T V^T = A exactly."""
    _say("zero", prec, k, p)
    A = np.zeros((50, 30), dtype=np.float64 if prec == "f64" else np.float32)
    U, T, V, piv, info = _run(ctx, A, k, p, 1, 1, prec, "auto")
    ref = corutv(A.astype(np.float64), k, p, 1, seed=1)
    assert info["qr_fallbacks"] >= 1
    assert info["rel_err"] == 0.0
    assert np.all(T == 0)
    np.testing.assert_array_equal(piv, ref["piv"])
    tol = 1e-13 if prec == "f64" else 1e-6
    ell = k + p
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= tol
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= tol


@pytest.mark.parametrize("prec", ["f64", "f32", "bf16x3", "bf16"])
@pytest.mark.parametrize("m,n,rank,k", [(3000, 2000, 30, 80), (900, 5000, 20, 100)])
def test_wide_sketch_breakdown_fp32_storage(ctx, prec, m, n, rank, k):
    """An exactly rank-`rank` matrix with l = k + 10 > 64: in F64 and F32 every
    sketch is numerically rank-deficient, so the CholeskyQR of the general
    form breaks down and the LDS or device-memory Householder tree (l > 64)
    takes over (F32 storage of the bases included); in the BF16 forms the
    rounding of A to bf16 may leave the sketches full rank.  Every form:
    finite, orthonormal bases and the matrix reproduced to its rounding."""
    _say("wide-sketch breakdown", prec, m, n, rank, k)
    rng = np.random.default_rng(m + n + rank)
    A64 = rng.standard_normal((m, rank)) @ rng.standard_normal((rank, n))
    A = A64 if prec == "f64" else A64.astype(np.float32)
    U, T, V, piv, info = _run(ctx, A, k, 10, 1, 9, prec, "auto")
    ell = k + 10
    if prec in ("f64", "f32"):
        assert info["qr_fallbacks"] >= 1
    print("fallbacks", info["qr_fallbacks"])
    assert np.all(np.isfinite(U)) and np.all(np.isfinite(V)) and np.all(np.isfinite(T))
    tol = 1e-13 if prec == "f64" else 1e-5
    assert np.max(np.abs(U.T @ U - np.eye(ell))) <= tol
    assert np.max(np.abs(V.T @ V - np.eye(ell))) <= tol
    bar = 1e-12 if prec == "f64" else (2e-3 if prec == "bf16" else 1e-5)
    assert np.linalg.norm(A.astype(np.float64) - U @ T @ V.T) <= bar * np.linalg.norm(A64)
