"""GPU parity of the single steps, through the C ABI, against the oracle.

* Gaussian test matrix: bit-identical to the oracle's stream (F64), F32 is its
  round-to-nearest-even.
* Passes over A (Y = A X, Z = A^T X): F64 within 1e-13 relative, F32 within
  the FP32 accumulation bound, both layouts, ragged and misaligned sizes.
* Thin QR (CholeskyQR2 / Householder fallback): equal to the oracle's
  Householder Q (unique with diag R > 0) within 1e-12; orthonormal to 1e-13.
* QRCP of the core, fed the oracle's input bits: the kernel's pivots are the
  oracle's at every step not decided by a near tie (margin rule), and its
  factorization is exact to rounding.
"""
import numpy as np
import pytest
import torch

from oracle.corutv import corutv
from oracle.dense import householder_qr, qrcp
from oracle.philox import omega
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


@pytest.mark.parametrize("n,ell,seed,sub", [(1000, 37, 1, 0), (4097, 16, 2**63 + 5, 3), (3, 1, 0, 0xFFFF),
                                            (200003, 64, 12345, 0)])
def test_omega_bit_exact(ctx, n, ell, seed, sub):
    _say("omega", n, ell, seed, sub)
    g = ctx.omega(n, ell, seed, sub).cpu().numpy()
    o = omega(n, ell, seed, sub)
    assert np.array_equal(g.view(np.uint64), o.view(np.uint64)), np.argwhere(g != o)[:5]
    g32 = ctx.omega(n, ell, seed, sub, torch.float32).cpu().numpy()
    assert np.array_equal(g32.view(np.uint32), o.astype(np.float32).view(np.uint32))


CASES = [
    # m, n, ell, layout, prec
    (1000, 777, 37, "row", "f64"), (1000, 777, 37, "col", "f64"), (1000, 777, 37, "row", "f32"),
    (1000, 777, 37, "col", "f32"), (513, 2050, 16, "row", "f32"), (4096, 1024, 112, "row", "f32"),
    (4096, 1024, 112, "col", "f64"), (3000, 700, 256, "row", "f32"), (1537, 1201, 1, "row", "f64"),
    (64, 64, 64, "col", "f32"), (300, 20000, 10, "row", "f32"), (2048, 1000, 200, "row", "f64"),
    # short output, long contraction: many partial slots per output tile, so
    # several threads share each entry of the partial sum
    (300, 40000, 10, "col", "f64"), (40000, 200, 20, "row", "f32"),
]


@pytest.mark.parametrize("m,n,ell,layout,prec", CASES)
@pytest.mark.parametrize("trans", [False, True])
def test_sketch_pass(ctx, m, n, ell, layout, prec, trans):
    _say("sketch", m, n, ell, layout, prec, trans)
    dt = np.float64 if prec == "f64" else np.float32
    rng = np.random.default_rng(m * 7 + n + ell)
    A = rng.standard_normal((m, n)).astype(dt)
    X = rng.standard_normal((m if trans else n, ell)).astype(dt)
    At = torch.from_numpy(A).cuda()
    if layout == "col":
        At = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    Y = ctx.sketch(At, torch.from_numpy(X).cuda(), trans=trans, prec=prec).cpu().numpy()
    ref = (A.astype(np.float64).T if trans else A.astype(np.float64)) @ X.astype(np.float64)
    K = m if trans else n
    scale = np.sqrt(K) * np.abs(X).max() * np.abs(A).max()
    tol = 1e-14 * np.sqrt(K) if prec == "f64" else 2e-6 * np.sqrt(K)
    err = np.max(np.abs(Y - ref)) / scale
    assert err <= tol, err


@pytest.mark.parametrize("rows,ell", [(5000, 40), (20000, 112), (777, 1), (3001, 130), (4000, 220)])
def test_tsqr_matches_householder(ctx, rows, ell):
    _say("tsqr", rows, ell)
    rng = np.random.default_rng(rows + ell)
    X = rng.standard_normal((rows, ell)) @ np.diag(np.logspace(0, -3, ell))
    Q, R, fb = ctx.tsqr(torch.from_numpy(X).cuda())
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = householder_qr(X)
    assert not fb
    assert np.max(np.abs(Q.T @ Q - np.eye(ell))) <= 1e-13 * max(1, ell / 32)
    assert np.max(np.abs(Q - Qo)) <= 1e-10
    assert np.max(np.abs(R - Ro)) <= 1e-12 * np.abs(Ro).max()
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) > 0)


@pytest.mark.parametrize("rows,ell,rank", [(3000, 30, 12), (2000, 64, 1), (500, 17, 16), (76800, 10, 5),
                                           (20037, 110, 60), (200, 48, 10), (250, 40, 5), (700, 16, 3)])
def test_tsqr_rank_deficient_falls_back(ctx, rows, ell, rank):
    """Cholesky breaks down; Householder QR gives an orthonormal Q with X = QR:
    the register-resident kernels (one workgroup: 500x17, 200x48, 250x40,
    700x16; the two-level tree with the rows split evenly: 3000x30,
    76800x10), the device-memory tree (panels of max(256, 4 ell,
    sqrt(rows ell)) rows, the last one ragged: 2000x64, 20037x110).  The
    first `rank` columns of X are independent, so Q[:, :rank] and R[:rank]
    are unique and equal the oracle's."""
    _say("tsqr-deficient", rows, ell, rank)
    rng = np.random.default_rng(rows)
    X = rng.standard_normal((rows, rank)) @ rng.standard_normal((rank, ell))
    Q, R, fb = ctx.tsqr(torch.from_numpy(X).cuda())
    Q, R = Q.cpu().numpy(), R.cpu().numpy()
    Qo, Ro = householder_qr(X)
    assert fb
    assert np.max(np.abs(Q.T @ Q - np.eye(ell))) <= 1e-13 * max(1, ell / 32)
    assert np.max(np.abs(Q @ R - X)) <= 1e-13 * np.abs(X).max() * np.sqrt(rows)
    assert np.all(np.diag(R) >= 0)
    assert np.all(np.tril(R, -1) == 0)
    assert np.max(np.abs(Q[:, :rank] - Qo[:, :rank])) <= 1e-10
    assert np.max(np.abs(R[:rank] - Ro[:rank])) <= 1e-11 * np.abs(Ro).max()


def _cores():
    out = []
    A = noisy_low_rank(400, 300, 20, 1e-6, seed=1)
    out.append(("c1-like", corutv(A, 20, 10, 1, seed=1)["D"]))
    rng = np.random.default_rng(5)
    for ell in (10, 30, 110, 128, 129, 150, 180, 192, 193, 200, 220, 224, 225, 256):
        out.append(("gauss%d" % ell, rng.standard_normal((ell, ell)) * np.logspace(0, -8, ell)))
    D = rng.standard_normal((40, 6)) @ rng.standard_normal((6, 40))
    out.append(("rank6", D))
    Z = np.zeros((12, 12))
    Z[:, 3] = 1.0
    Z[:, 7] = 1.0
    out.append(("ties", Z))
    return out


@pytest.mark.parametrize("name,D", _cores(), ids=[c[0] for c in _cores()])
def test_qrcp_pivots_margin_rule(ctx, name, D):
    """Identical input bits: the kernel sums column norms in its own fixed
    order (partial sums per lane and across the four lanes of a column, fused
    multiply-adds), the oracle sequentially, so norms differ by rounding.  The
    kernel's pivot sequence is replayed in the oracle's arithmetic; at every
    step its choice must be the oracle's largest norm unless the two norms are
    within tau = 8 l u max_j ||D_j|| (near ties are listed, not failed).
    When the sequences agree, R and Qt agree to the rounding of the
    factorization."""
    from tests.pivots import margin_tau, pivot_margins

    _say("qrcp", name, D.shape)
    Qt, R, piv = ctx.qrcp(torch.from_numpy(np.ascontiguousarray(D)).cuda())
    Qt, R, piv = Qt.cpu().numpy(), R.cpu().numpy(), piv.cpu().numpy()
    tau = margin_tau(D)
    near = pivot_margins(D, piv, tau)
    print("near-tie steps (step, norm gap):", near, "tau %.3e" % tau)
    Qto, Ro, pivo = qrcp(D)
    ell = D.shape[0]
    scale = max(1.0, np.abs(D).max())
    # the kernel's own factorization is exact to rounding whatever the pivots
    assert np.max(np.abs(Qt @ R - D[:, piv])) <= 1e-13 * ell * scale
    assert np.max(np.abs(Qt.T @ Qt - np.eye(ell))) <= 1e-14 * ell
    assert np.all(np.tril(R, -1) == 0) and np.all(np.diag(R) >= 0)
    if np.array_equal(piv, pivo):
        np.testing.assert_allclose(R, Ro, rtol=0, atol=1e-13 * ell * scale)
        if name != "rank6" and name != "ties":  # trailing reflectors of a zero block are arbitrary
            np.testing.assert_allclose(Qt, Qto, rtol=0, atol=1e-10)
    else:
        assert near, "pivots differ although no step is a near tie"


BF_CASES = [
    (1000, 777, 37, "row"), (1000, 777, 37, "col"), (3000, 2048, 220, "row"), (4096, 1000, 112, "col"),
    (300, 20000, 10, "row"), (513, 2050, 16, "row"),
]


@pytest.mark.parametrize("m,n,ell,layout", BF_CASES)
@pytest.mark.parametrize("trans", [False, True])
@pytest.mark.parametrize("prec", ["bf16", "bf16x3"])
def test_sketch_pass_bf16_forms(ctx, m, n, ell, layout, trans, prec):
    """BF16: operands rounded to nearest-even bfloat16, FP32 accumulation.
    BF16X3: lo*hi + hi*lo + hi*hi of the 2-way split.  The reference is the
    exact (float64) product of the same rounded operands (oracle.bf16)."""
    from oracle.bf16 import matmul_bf16, matmul_bf16x3

    _say("sketch", prec, m, n, ell, layout, trans)
    rng = np.random.default_rng(m + 3 * n + ell)
    A = rng.standard_normal((m, n)).astype(np.float32)
    X = rng.standard_normal((m if trans else n, ell)).astype(np.float32)
    At = torch.from_numpy(A).cuda()
    if layout == "col":
        At = torch.from_numpy(np.ascontiguousarray(A.T)).cuda().t()
    Y = ctx.sketch(At, torch.from_numpy(X).cuda(), trans=trans, prec=prec).cpu().numpy()
    Aop = A.T if trans else A
    ref = (matmul_bf16 if prec == "bf16" else matmul_bf16x3)(Aop, X)
    K = Aop.shape[1]
    scale = np.sqrt(K) * np.abs(X).max() * np.abs(A).max()
    err = np.max(np.abs(Y - ref)) / scale
    assert err <= 2e-6 * np.sqrt(K), err
    # and it is not the float32 product: bf16 rounding is visible
    exact = Aop.astype(np.float64) @ X.astype(np.float64)
    if prec == "bf16":
        assert np.max(np.abs(Y - exact)) / scale > 1e-4
