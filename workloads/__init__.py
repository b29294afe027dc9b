"""Seeded synthetic inputs shaped like the paper's workloads.

This module holds no CoR-UTV arithmetic: it only draws input matrices, with
numpy's PCG64 generator (``numpy.random.default_rng(seed)``), so that the
oracle and the GPU library consume identical bits.  (The method's own random
test matrix is *not* drawn here; both sides regenerate it from the Philox
stream definition.)

Shapes and structure:

* ``noisy_low_rank``  -- A = X Y^T + eps N with Gaussian X (m x k), Y (n x k),
  N (m x n): an exactly rank-k matrix plus small noise (plain CoR-UTV runs).
* ``decaying``        -- A = U0 diag(sigma) V0^T + eps N with Haar-orthonormal
  U0, V0 (QR of Gaussians, positive diagonal), sigma_i = exp(-i/tau)
  ("exp") or i^-alpha ("poly").
* ``sec51_matrix``    -- the Sec. 5.1 test matrix: random orthonormal factors,
  k singular values decreasing linearly from 1 to 1e-9, the rest zero, plus
  0.1 sigma_k E with E a Gaussian matrix normalised to unit spectral norm.
* ``low_rank_plus_sparse`` -- M = X Y^T + S (robust PCA): Gaussian factors and
  a sparse S on a uniformly drawn support (without replacement) whose values
  are either uniform in [-amp, amp] or drawn from {-amp, +amp} (Table 1).
* ``serving_requests`` -- a Poisson stream of decomposition requests with
  log-uniform m, n, uniform k, sigma_i = exp(-i/k) truncated at 1e-4.
* ``serving_pool`` / ``serving_stream`` -- the same distributions split into
  a pool of distinct request matrices (shape and rank) and a Poisson stream
  of requests that each pick a pool entry, q, a precision tag and a seed.
"""
import numpy as np


def _rng(seed):
    return np.random.default_rng(seed)


def haar(rng, rows, cols, dtype=np.float64):
    G = rng.standard_normal((rows, cols))
    Q, R = np.linalg.qr(G)
    s = np.sign(np.diag(R))
    s[s == 0] = 1.0
    return (Q * s).astype(dtype, copy=False)


def noisy_low_rank(m, n, k, eps, seed, dtype=np.float64):
    rng = _rng(seed)
    X = rng.standard_normal((m, k))
    Y = rng.standard_normal((n, k))
    A = X @ Y.T
    if eps:
        A += eps * rng.standard_normal((m, n))
    return A.astype(dtype, copy=False)


def decaying(m, n, r, eps, seed, kind="exp", tau=25.0, alpha=1.5, dtype=np.float64):
    rng = _rng(seed)
    U0 = haar(rng, m, r)
    V0 = haar(rng, n, r)
    i = np.arange(1, r + 1, dtype=np.float64)
    sig = np.exp(-i / tau) if kind == "exp" else i ** (-alpha)
    A = (U0 * sig) @ V0.T
    if eps:
        if dtype == np.float32:
            A = A.astype(np.float32)
            A += np.float32(eps) * rng.standard_normal((m, n), dtype=np.float32)
            return A
        A += eps * rng.standard_normal((m, n))
    return A.astype(dtype, copy=False)


def sec51_matrix(n, k, seed):
    rng = _rng(seed)
    U = haar(rng, n, k)
    V = haar(rng, n, k)
    sig = np.linspace(1.0, 1e-9, k)
    E = rng.standard_normal((n, n))
    E /= np.linalg.norm(E, 2)
    return (U * sig) @ V.T + 0.1 * sig[-1] * E, sig


def low_rank_plus_sparse(m, n, r, frac, amp, seed, values="uniform", dtype=np.float64, grid=None):
    """Returns (M, L, S).

    grid: if given (e.g. 2**-6), the Gaussian factors and the corruption values
    are rounded to multiples of it, so that M = L + S holds exactly in float32
    (products and sums stay within 24 significant bits for the sizes used):
    float32 data is then exactly low-rank plus sparse."""
    rng = _rng(seed)
    X = rng.standard_normal((m, r))
    Y = rng.standard_normal((n, r))
    if grid:
        X = np.round(X / grid) * grid
        Y = np.round(Y / grid) * grid
    L = X @ Y.T
    count = int(round(frac * m * n))
    pos = rng.choice(m * n, size=count, replace=False)
    if values == "uniform":
        vals = rng.uniform(-amp, amp, size=count)
    else:
        vals = amp * rng.choice(np.array([-1.0, 1.0]), size=count)
    if grid:
        vals = np.round(vals / grid) * grid
        vals[vals == 0] = grid
    S = np.zeros(m * n)
    S[pos] = vals
    S = S.reshape(m, n)
    M = L + S
    return M.astype(dtype), L.astype(dtype), S.astype(dtype)


def serving_requests(count, seed, m_range=(1000, 40000), n_range=(500, 20000),
                     k_range=(5, 150), p=10, qps=100.0):
    """List of dicts {t_arrival, m, n, k, p, q, prec, seed} for a Poisson stream."""
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=count))
    m = np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1]), size=count)).astype(int)
    n = np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]), size=count)).astype(int)
    k = rng.integers(k_range[0], k_range[1] + 1, size=count)
    q = rng.integers(1, 3, size=count)
    prec = rng.choice(np.array(["f64", "bf16"]), size=count)
    om = rng.integers(0, 2**62, size=count)
    out = []
    for i in range(count):
        kk = int(min(k[i], min(m[i], n[i]) - p))
        out.append(dict(t_arrival=float(t[i]), m=int(m[i]), n=int(n[i]), k=kk, p=p,
                        q=int(q[i]), prec=str(prec[i]), seed=int(om[i])))
    return out


def serving_matrix(m, n, k, seed, dtype=np.float64):
    """sigma_i = exp(-i/k) for i <= min(ceil(9.2 k), min(m, n) // 2), plus 1e-4 noise."""
    r = int(min(np.ceil(9.2 * k), min(m, n) // 2))
    return decaying(m, n, r, 1e-4, seed, kind="exp", tau=float(k), dtype=dtype)


def serving_pool(count, seed, m_range=(1000, 40000), n_range=(500, 20000), k_range=(5, 150), p=10):
    """count distinct request shapes: list of dicts {m, n, k, r} with m, n
    log-uniform, k uniform, r = min(ceil(9.2 k), min(m, n) // 2) decaying
    singular values (exp(-i/k) down to 1e-4)."""
    rng = _rng(seed)
    out = []
    for _ in range(count):
        m = int(np.exp(rng.uniform(np.log(m_range[0]), np.log(m_range[1]))))
        n = int(np.exp(rng.uniform(np.log(n_range[0]), np.log(n_range[1]))))
        k = int(rng.integers(k_range[0], k_range[1] + 1))
        k = int(min(k, min(m, n) - p))
        r = int(min(np.ceil(9.2 * k), min(m, n) // 2))
        out.append(dict(m=m, n=n, k=k, r=r))
    return out


def serving_stream(count, pool_size, qps, seed, tags=("f64", "bf16")):
    """Poisson arrivals at rate qps: list of dicts {t, entry, q, tag, seed}."""
    rng = _rng(seed)
    t = np.cumsum(rng.exponential(1.0 / qps, size=count))
    entry = rng.integers(0, pool_size, size=count)
    q = rng.integers(1, 3, size=count)
    tag = rng.integers(0, len(tags), size=count)
    om = rng.integers(0, 2**62, size=count)
    return [dict(t=float(t[i]), entry=int(entry[i]), q=int(q[i]), tag=tags[int(tag[i])], seed=int(om[i]))
            for i in range(count)]
