"""Small dense factorizations used by CoR-UTV (float64, plain numpy).

* ``householder_qr`` -- the "QR decomposition" of the sketches (eq. 6,
  Algorithm 1 step "Compute QR decompositions").  The paper does not fix the
  sign convention; the factor is normalised to diag(R) >= 0, which makes Q
  unique for full-column-rank input.
* ``qrcp`` -- the QR with column pivoting of the l x l core (eq. 8), Businger &
  Golub's greedy rule: at each step move the trailing column of largest
  Euclidean norm to the front, then annihilate it below the diagonal with a
  Householder reflector.  Norms are recomputed from scratch at every step (no
  downdating), ties go to the lowest current column position, and diag(R) is
  made non-negative at the end.  Every reduction is a sequential sum in row
  order of separately rounded products, so that the pivot sequence is a
  deterministic function of the input bits.  An implementation that sums in
  another order sees norms that differ by rounding; its pivots are compared
  with these by replaying them (``follow``) and bounding, at every step, how
  far its choice falls short of the largest norm.
* ``jacobi_svd`` -- one-sided (Hestenes) Jacobi SVD, used only by the pins to
  get singular values (Eckart-Young optimum of eq. 3, interlacing checks).
"""
import numpy as np


def householder_qr(X):
    """Thin QR X = Q R of an m x l matrix (m >= l) by Householder reflectors.

    Returns (Q m x l with orthonormal columns, R l x l upper triangular with
    non-negative diagonal).  A column that is exactly zero below the diagonal
    gets no reflector (R[s, s] = 0) and Q keeps the corresponding unit vector,
    so Q stays orthonormal for rank-deficient X as well.
    """
    W = np.array(X, dtype=np.float64, copy=True)
    m, l = W.shape
    if m < l:
        raise ValueError("householder_qr needs m >= l")
    vs = []
    for s in range(l):
        x = W[s:, s]
        nrm = np.sqrt(np.dot(x, x))
        if nrm == 0.0:
            vs.append(None)
            continue
        alpha = -nrm if x[0] >= 0 else nrm
        v = x.copy()
        v[0] = x[0] - alpha
        tau = 2.0 / np.dot(v, v)
        W[s:, s + 1:] -= np.outer(v, tau * (v @ W[s:, s + 1:]))
        W[s, s] = alpha
        W[s + 1:, s] = 0.0
        vs.append((v, tau))
    R = np.triu(W[:l, :])
    # Q = H_0 H_1 ... H_{l-1} applied to the first l columns of the identity.
    Q = np.zeros((m, l))
    Q[np.arange(l), np.arange(l)] = 1.0
    for s in range(l - 1, -1, -1):
        if vs[s] is None:
            continue
        v, tau = vs[s]
        Q[s:, :] -= np.outer(v, tau * (v @ Q[s:, :]))
    neg = np.diag(R) < 0
    R[neg, :] *= -1.0
    Q[:, neg] *= -1.0
    return Q, R


def qrcp(D, follow=None, trace=None):
    """Column-pivoted QR of a square matrix: D[:, piv] = Qt @ R (eq. 8).

    Returns (Qt orthogonal, R upper triangular with diag >= 0 and
    |R[0,0]| >= |R[1,1]| >= ..., piv int32 with D[:, piv] = Qt R).

    Businger-Golub: at step s the trailing column of largest Euclidean norm
    is swapped to position s and a Householder reflector annihilates it below
    the diagonal.  The arithmetic is the plain one, in a fixed order:
      norms:  acc_j = 0; for i = s..l-1: acc_j = acc_j + W[i,j]*W[i,j]
      pivot:  first j >= s with the largest acc_j (ties: lowest position)
      reflector on x = W[s:, s] (after the swap): nrm = sqrt(acc_p);
              alpha = -nrm if x0 >= 0 else nrm; v = x with v0 = x0 - alpha;
              vtv = sequential sum of v_i*v_i; tau = 2 / vtv
      update: d_j = sequential sum over i of v_i*W[s+i,j]; f_j = d_j*tau;
              W[s+i,j] = W[s+i,j] - f_j*v_i
    Qt = H_0 H_1 ... H_{l-1} (H_s = I - tau_s v_s v_s^T) is formed after the
    loop; it does not influence the pivots.

    follow: optional sequence of original column indices.  At step s the
    column D[:, follow[s]] is taken instead of the argmax (every other step
    of the arithmetic is unchanged).  This replays another implementation's
    pivot sequence so that, at every step, its choice can be compared with
    the largest norm this arithmetic sees.
    trace: optional list; for every step the tuple (acc, chosen position - s)
    is appended, acc being the squared norms of the trailing columns
    (positions s..l-1) before the swap.
    """
    W = np.array(D, dtype=np.float64, copy=True)
    l = W.shape[0]
    if W.shape != (l, l):
        raise ValueError("qrcp expects a square matrix")
    piv = np.arange(l, dtype=np.int32)
    reflectors = []
    for s in range(l):
        acc = np.zeros(l - s)
        for i in range(s, l):
            acc = acc + W[i, s:] * W[i, s:]
        if follow is None:
            p = s + int(np.argmax(acc))
        else:
            where = np.nonzero(piv[s:] == int(follow[s]))[0]
            if where.size != 1:
                raise ValueError("follow is not a permutation of the column indices")
            p = s + int(where[0])
        if trace is not None:
            trace.append((acc.copy(), p - s))
        if p != s:
            W[:, [s, p]] = W[:, [p, s]]
            piv[[s, p]] = piv[[p, s]]
        nrm = np.sqrt(acc[p - s])
        if nrm == 0.0:
            continue  # trailing block is exactly zero: H = I
        x0 = W[s, s]
        alpha = -nrm if x0 >= 0 else nrm
        v = W[s:, s].copy()
        v[0] = x0 - alpha
        vtv = 0.0
        for vi in v:
            vtv = vtv + vi * vi
        tau = 2.0 / vtv
        if s + 1 < l:
            d = np.zeros(l - s - 1)
            for i in range(l - s):
                d = d + v[i] * W[s + i, s + 1:]
            f = d * tau
            for i in range(l - s):
                W[s + i, s + 1:] = W[s + i, s + 1:] - f * v[i]
        W[s, s] = alpha
        W[s + 1:, s] = 0.0
        reflectors.append((s, v, tau))
    Qt = np.eye(l)
    for s, v, tau in reversed(reflectors):  # Qt = H_0 (H_1 (... H_{l-1}))
        Qt[s:, :] -= np.outer(v, tau * (v @ Qt[s:, :]))
    R = np.triu(W)
    neg = np.diag(R) < 0
    R[neg, :] = -R[neg, :]
    Qt[:, neg] = -Qt[:, neg]
    return Qt, R, piv


def _round_robin(n):
    """Brent-Luk tournament: n-1 rounds of disjoint index pairs covering all pairs."""
    idx = list(range(n + (n % 2)))
    k = len(idx)
    rounds = []
    for _ in range(k - 1):
        pairs = [(idx[i], idx[k - 1 - i]) for i in range(k // 2)]
        rounds.append([(min(a, b), max(a, b)) for a, b in pairs if a < n and b < n])
        idx = [idx[0]] + [idx[-1]] + idx[1:-1]
    return rounds


def jacobi_svd(A, max_sweeps=80):
    """Singular values (descending) and right/left vectors by one-sided Jacobi.

    Columns are orthogonalised pairwise by plane rotations until every pair
    satisfies |a_p . a_q| <= n * eps * |a_p| |a_q|.  Returns (U, s, V) with
    A = U diag(s) V^T (thin).
    """
    A = np.array(A, dtype=np.float64, copy=True)
    transposed = A.shape[0] < A.shape[1]
    if transposed:
        A = A.T.copy()
    m, n = A.shape
    V = np.eye(n)
    tol = n * np.finfo(np.float64).eps
    rounds = _round_robin(n)
    for _ in range(max_sweeps):
        rotated = False
        for pairs in rounds:
            if not pairs:
                continue
            p = np.array([a for a, _ in pairs])
            q = np.array([b for _, b in pairs])
            ap, aq = A[:, p], A[:, q]
            alpha = np.einsum("ij,ij->j", ap, ap)
            beta = np.einsum("ij,ij->j", aq, aq)
            gamma = np.einsum("ij,ij->j", ap, aq)
            act = np.abs(gamma) > tol * np.sqrt(alpha * beta)
            if not np.any(act):
                continue
            rotated = True
            zeta = np.where(act, (beta - alpha) / (2.0 * np.where(act, gamma, 1.0)), 0.0)
            t = np.where(act, np.sign(zeta + (zeta == 0)) / (np.abs(zeta) + np.sqrt(1.0 + zeta * zeta)), 0.0)
            c = 1.0 / np.sqrt(1.0 + t * t)
            s = c * t
            A[:, p], A[:, q] = c * ap - s * aq, s * ap + c * aq
            vp, vq = V[:, p], V[:, q]
            V[:, p], V[:, q] = c * vp - s * vq, s * vp + c * vq
        if not rotated:
            break
    sig = np.sqrt(np.einsum("ij,ij->j", A, A))
    order = np.argsort(-sig, kind="stable")
    sig = sig[order]
    V = V[:, order]
    U = A[:, order] / np.where(sig > 0, sig, 1.0)
    if transposed:
        return V, sig, U
    return U, sig, V
