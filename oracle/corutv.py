"""CoR-UTV in float64 (Sec. 3.1, eqs. 4-9, Algorithm 1).

``corutv`` follows the paper's steps in its order:

1. Draw the n x l standard Gaussian test matrix (``oracle.philox.omega``).
2. Sketch the column space, C1 = A Psi (eq. 4), and the row space,
   C2 = A^T C1 (eq. 5); with q power iterations (Algorithm 1) the pair of
   products is repeated q + 1 times.
3. Thin QR of both sketches, C1 = Q1 R1, C2 = Q2 R2 (eq. 6).
4. Core D = Q1^T A Q2 (eq. 7), an l x l matrix, formed as Q1^T (A Q2).
5. QRCP of the core, D P = Qt R (eq. 8).
6. U = Q1 Qt, T = R, V = Q2 P (eq. 9) -- V's column j is Q2's column piv[j].

Two arithmetic forms of steps 2-3 are provided:

* ``mode="literal"``: Algorithm 1 as printed -- the power products without
  re-orthonormalisation, QR only at the end.  In floating point the sketch's
  condition number grows like (s1/sl)^(2q+1), so this is kept for the
  equivalence pin only.
* ``mode="stabilized"`` (default): Q1 = qf(A Psi); q times { W = qf(A^T Q1);
  Q1 = qf(A W) }; Z = A^T Q1; Q2, R_Z = qf(Z).  With qf the Q factor of a
  thin QR with positive diagonal, qf(X G) = qf(X) for any upper triangular G
  with positive diagonal, so each re-orthonormalised iterate spans exactly the
  literal one and the returned Q1, Q2 are those of Algorithm 1 in exact
  arithmetic.

Orientation (Sec. 3 opening): for m >= n the paper's T is upper triangular;
for m < n the method runs on A^T and transposes back, giving a lower
triangular T.  ``tri`` selects the triangle explicitly: "lower" for m >= n
runs the QRCP on D^T, so D = P R^T Qt^T and U = Q1 P, T = R^T, V = Q2 Qt.
"""
import numpy as np

from .dense import householder_qr, qrcp
from .philox import omega


def _qf(X):
    return householder_qr(X)[0]


def corutv(A, k, p, q, seed, tri="auto", sub=0, mode="stabilized", core="pass"):
    """Rank-l CoR-UTV of A (l = k + p).  Returns a dict with U, T, V, piv and
    the intermediates Omega, Q1, Q2, D (and R_Z in stabilized mode).

    core: "pass" forms D = Q1^T (A Q2) (eq. 7, one more product with A);
    "rz" (stabilized mode) takes D = R_Z^T from the QR of the second sketch
    Z = A^T Q1 = Q2 R_Z, since then Q1^T A Q2 = (A^T Q1)^T Q2 = R_Z^T Q2^T Q2;
    "approx" is the single-revisit core of Sec. 3.1 and Algorithm 1,
    D_approx = Q1^T C1 (Q2^T Psi)^+, with C1 = A Psi the last product with A
    and Psi the matrix it was formed from (Omega when q = 0, else the last
    power iterate; the C2 that produced the last C1).  It equals D when
    A = A Q2 Q2^T."""
    A = np.asarray(A, dtype=np.float64)
    m, n = A.shape
    ell = k + p
    if k < 1 or p < 0 or q < 0 or ell > min(m, n):
        raise ValueError("need k >= 1, p >= 0, q >= 0, k + p <= min(m, n)")
    if tri == "auto":
        tri = "upper" if m >= n else "lower"
    if tri not in ("upper", "lower"):
        raise ValueError("tri must be auto, upper or lower")
    if m < n:
        inner = corutv(A.T, k, p, q, seed, tri="lower" if tri == "upper" else "upper",
                       sub=sub, mode=mode, core=core)
        out = dict(inner)
        out.update(U=inner["V"], T=inner["T"].T.copy(), V=inner["U"], transposed=True)
        return out

    Om = omega(n, ell, seed, sub)
    res = {"Omega": Om, "transposed": False, "tri": tri}
    if mode == "literal":
        C2 = Om
        for _ in range(q + 1):
            Psi = C2
            C1 = A @ C2
            C2 = A.T @ C1
        Q1, R1 = householder_qr(C1)
        Q2, R2 = householder_qr(C2)
        res.update(C1=C1, C2=C2, R1=R1, R2=R2)
    elif mode == "stabilized":
        Psi = Om
        C1 = A @ Psi
        Q1 = _qf(C1)
        for _ in range(q):
            Psi = _qf(A.T @ Q1)
            C1 = A @ Psi
            Q1 = _qf(C1)
        Z = A.T @ Q1
        Q2, RZ = householder_qr(Z)
        res.update(Z=Z, R_Z=RZ)
    else:
        raise ValueError("mode must be literal or stabilized")

    if core == "pass":
        D = Q1.T @ (A @ Q2)
    elif core == "rz" and mode == "stabilized":
        D = res["R_Z"].T.copy()
    elif core == "approx":
        D = Q1.T @ C1 @ np.linalg.pinv(Q2.T @ Psi)
        res.update(Psi=Psi)
    else:
        raise ValueError("core must be pass, approx, or rz in stabilized mode")
    if tri == "upper":
        Qt, R, piv = qrcp(D)
        U, T, V = Q1 @ Qt, R, Q2[:, piv]
    else:
        Qt, R, piv = qrcp(D.T.copy())
        U, T, V = Q1[:, piv], R.T.copy(), Q2 @ Qt
    res.update(Q1=Q1, Q2=Q2, D=D, Qt=Qt, R=R, piv=piv, U=U, T=T, V=V)
    return res


def reconstruct(U, T, V):
    return U @ T @ V.T


def rel_err(A, U, T, V):
    """Relative Frobenius error ||A - U T V^T||_F / ||A||_F, formed explicitly."""
    A = np.asarray(A, dtype=np.float64)
    E = A - reconstruct(U, T, V)
    return np.sqrt(np.sum(E * E)) / np.sqrt(np.sum(A * A))


def truncate(U, T, V, r, tri="upper"):
    """Rank-r approximation from a rank-l CoR-UTV (Sec. 5.2 and eq. 12).

    Upper T: U(:, 1:r) T(1:r, :) V^T, the row truncation of eq. 12.  A lower T
    comes from the transposed problem, whose row truncation becomes the
    column truncation U T(:, 1:r) V(:, 1:r)^T here.
    """
    if r <= 0:
        return np.zeros((U.shape[0], V.shape[0]))
    if tri == "upper":
        return U[:, :r] @ T[:r, :] @ V.T
    return U @ T[:, :r] @ V[:, :r].T
