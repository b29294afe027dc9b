"""ALM-CoRUTV robust PCA (Sec. 4, Algorithm 2), float64.

Solves min ||L||_* + lambda ||S||_1 s.t. M = L + S (eq. 11) by the inexact
augmented Lagrange multiplier iteration, with CoR-UTV thresholding as the
low-rank step:

  B_j     = M - S_j + Y_j / mu_j
  L_{j+1} = C_{1/mu_j}(B_j)            (eq. 12: U(:,1:r) T(1:r,:) V^T, r = number
                                        of diagonal entries of T above 1/mu_j)
  S_{j+1} = shrink_{lambda/mu_j}(M - L_{j+1} + Y_j / mu_j)
  Y_{j+1} = Y_j + mu_j (M - L_{j+1} - S_{j+1})
  mu_{j+1} = min(rho mu_j, mu_bar)

Readings of points the paper leaves open:
* the S step uses Y_j (the multiplier of the current iterate);
* the printed mu update takes a max, which would freeze mu after one step
  while the text says the continuation increases mu; min (capped growth) is
  used;
* mu_0, rho and mu_bar are "as suggested" by the inexact-ALM reference and not
  printed: mu_0 = 1.25 / ||M||_2 with ||M||_2 estimated by T[0, 0] of a
  CoR-UTV of M (same k, p, q, seed, sub = 0xFFFF), rho = 1.5,
  mu_bar = 1e7 mu_0; Y_0 = S_0 = 0 as printed;
* CoR-UTV iteration j draws its own test matrix (sub = j);
* "diagonals of T greater than delta": |T_ii| > delta strictly (T has a
  non-negative, non-increasing diagonal, so r is a prefix length).
"""
import numpy as np

from .corutv import corutv, truncate

SUB_NORM_ESTIMATE = 0xFFFF


def shrink(X, delta):
    """Shrinkage operator sgn(x) max(|x| - delta, 0), elementwise."""
    return np.sign(X) * np.maximum(np.abs(X) - delta, 0.0)


def threshold_rank(T, delta):
    d = np.abs(np.diag(T))
    return int(np.sum(d > delta))


def alm_corutv(M, k, p, q, seed, lam=None, max_iter=50, tol=0.0, rho=1.5,
               mu_bar_factor=1e7, mu0=None):
    """Returns (L, S, info) with info = {iters, zeta, ranks, mu, mu0}."""
    M = np.asarray(M, dtype=np.float64)
    m, n = M.shape
    if lam is None or lam <= 0:
        lam = 1.0 / np.sqrt(max(m, n))
    tri = "upper" if m >= n else "lower"
    if mu0 is None:
        est = corutv(M, k, p, q, seed, sub=SUB_NORM_ESTIMATE)
        mu0 = 1.25 / est["T"][0, 0]
    mu = mu0
    mu_bar = mu_bar_factor * mu0
    normM = np.sqrt(np.sum(M * M))
    S = np.zeros_like(M)
    Y = np.zeros_like(M)
    ranks, zetas = [], []
    L = np.zeros_like(M)
    it = 0
    for j in range(max_iter):
        B = M - S + Y / mu
        res = corutv(B, k, p, q, seed, sub=j)
        r = threshold_rank(res["T"], 1.0 / mu)
        L = truncate(res["U"], res["T"], res["V"], r, tri)
        S = shrink(M - L + Y / mu, lam / mu)
        Z = M - L - S
        Y = Y + mu * Z
        mu = min(rho * mu, mu_bar)
        zeta = np.sqrt(np.sum(Z * Z)) / normM
        ranks.append(r)
        zetas.append(zeta)
        it = j + 1
        if tol > 0 and zeta < tol:
            break
    return L, S, {"iters": it, "zeta": zetas[-1] if zetas else None, "zetas": zetas,
                  "ranks": ranks, "mu": mu, "mu0": mu0, "lam": lam}
