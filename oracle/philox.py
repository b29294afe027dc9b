"""Gaussian test matrix of CoR-UTV (Sec. 3.1; Algorithm 1, first step).

The paper only asks for a matrix with i.i.d. standard Gaussian entries drawn by
"a random number generator".  To let the GPU regenerate the very same matrix
(without ever shipping it), the stream is defined here from published pieces:

* Philox4x64-10 (Salmon, Moraes, Dror, Shaw, "Parallel random numbers: as easy
  as 1, 2, 3", SC'11): a 4x64-bit counter, a 2x64-bit key, 10 rounds, key
  bumped between rounds by the Weyl constants.
* Entry Omega[i, j] of an n x l test matrix uses counter (i, j, tag, sub) and
  key (seed, 0).  tag = 0 for the test matrix; ``sub`` separates independent
  draws (the ALM iteration index).  One normal per counter, so the matrix does
  not depend on n or l beyond its own index (columns are nested in l).
* Box-Muller (1958): z = sqrt(-2 ln u1) * cos(2 pi u2) with
  u1 = ((w0 >> 11) + 1) * 2^-53 in (0, 1] and u2 = (w1 >> 11) * 2^-53 in [0, 1).
* ln and cos are *defined* by the truncated series below, evaluated with plain
  IEEE-754 double operations (each multiply, add, divide and square root
  rounded to nearest, no fused multiply-add), so that any faithful
  implementation of the same definition produces identical bits:

  - ln u:  u = f * 2^e with f in [sqrt(1/2), sqrt(2)];  s = (f - 1) / (f + 1);
    ln f = 2 s * sum_{k=0}^{11} s^(2k) / (2k+1)  (Horner in s^2);
    ln u = e*LN2_HI + (e*LN2_LO + ln f), LN2_HI = ln 2 cut to 32 significant
    bits, LN2_LO = ln 2 - LN2_HI rounded.
  - cos(2 pi u2): exact quadrant reduction v = 4 u2, q = floor(v), f = v - q,
    then f -> 1 - f above 1/2 (exact); x = (pi/2) * g (one rounding) and
    cos x = sum_{k=0}^{9} (-1)^k x^(2k)/(2k)!,
    sin x = x * sum_{k=0}^{9} (-1)^k x^(2k)/(2k+1)!  (Horner in x^2),
    coefficients being the correctly rounded doubles of those rationals.

Pins: raw Philox words against numpy's independent Philox4x64-10; ln/cos/z
against libm within a few ulp; moments and a Kolmogorov-Smirnov test.
"""
from fractions import Fraction
from math import factorial

import numpy as np

# Philox4x64 constants (Salmon et al. 2011, Table 2 / Random123 distribution).
_M0 = np.uint64(0xD2E7470EE14C6C93)
_M1 = np.uint64(0xCA5A826395121157)
_W0 = np.uint64(0x9E3779B97F4A7C15)  # golden ratio
_W1 = np.uint64(0xBB67AE8584CAA73B)  # sqrt(3) - 1
_MASK32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

TAG_OMEGA = 0


def _mulhilo(a, b):
    """Full 64x64 -> 128-bit product, returned as (hi, lo) uint64 arrays."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    lo = a * b  # wraps mod 2^64
    a0, a1 = a & _MASK32, a >> _S32
    b0, b1 = b & _MASK32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _MASK32) + (p10 & _MASK32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, lo


def philox4x64_10(ctr, key):
    """Philox4x64 with 10 rounds.

    ctr: (..., 4) uint64 counters; key: (..., 2) uint64 keys (broadcastable).
    Returns (..., 4) uint64 output words.
    """
    ctr = np.array(ctr, dtype=np.uint64, copy=True)
    key = np.array(key, dtype=np.uint64, copy=True)
    c0, c1, c2, c3 = (np.atleast_1d(ctr[..., i]) for i in range(4))
    k0, k1 = np.atleast_1d(key[..., 0]), np.atleast_1d(key[..., 1])
    with np.errstate(over="ignore"):
        for r in range(10):
            if r > 0:  # key bump between rounds
                k0 = k0 + _W0
                k1 = k1 + _W1
            hi0, lo0 = _mulhilo(_M0, c0)
            hi1, lo1 = _mulhilo(_M1, c2)
            c0, c1, c2, c3 = hi1 ^ c1 ^ k0, lo1, hi0 ^ c3 ^ k1, lo0
    if ctr.ndim == 1:
        c0, c1, c2, c3 = c0[0], c1[0], c2[0], c3[0]
    return np.stack(np.broadcast_arrays(c0, c1, c2, c3), axis=-1)


# ---- transcendental pieces, defined by series (see module docstring) -------
_LN_COEF = [1.0 / (2 * k + 1) for k in range(12)]          # 1/(2k+1), k = 0..11
_COS_COEF = [float(Fraction((-1) ** k, factorial(2 * k))) for k in range(10)]
_SIN_COEF = [float(Fraction((-1) ** k, factorial(2 * k + 1))) for k in range(10)]
_LN2_HI = float.fromhex("0x1.62e42fee00000p-1")   # ln 2 to 32 significant bits
_LN2_LO = float.fromhex("0x1.a39ef35793c76p-33")  # ln 2 - LN2_HI, rounded
_HALF_PI = float.fromhex("0x1.921fb54442d18p+0")  # pi/2 rounded
_SQRT2 = float.fromhex("0x1.6a09e667f3bcdp+0")    # sqrt(2) rounded


def series_ln(u):
    """ln(u) for normal positive doubles u <= 1, by the atanh series."""
    u = np.asarray(u, dtype=np.float64)
    bits = u.view(np.uint64)
    e = ((bits >> np.uint64(52)) & np.uint64(0x7FF)).astype(np.int64) - 1023
    fbits = (bits & np.uint64(0x000FFFFFFFFFFFFF)) | np.uint64(0x3FF0000000000000)
    f = fbits.view(np.float64).copy()
    big = f > _SQRT2
    f[big] = f[big] * 0.5
    e = e + big.astype(np.int64)
    s = (f - 1.0) / (f + 1.0)
    s2 = s * s
    p = np.full_like(s, _LN_COEF[11])
    for k in range(10, -1, -1):
        p = p * s2 + _LN_COEF[k]
    lnf = 2.0 * (s * p)
    ef = e.astype(np.float64)
    return ef * _LN2_HI + (ef * _LN2_LO + lnf)


def _cos_sin_poly(x):
    x2 = x * x
    pc = np.full_like(x, _COS_COEF[9])
    ps = np.full_like(x, _SIN_COEF[9])
    for k in range(8, -1, -1):
        pc = pc * x2 + _COS_COEF[k]
        ps = ps * x2 + _SIN_COEF[k]
    return pc, x * ps


def series_cos_2pi(u2):
    """cos(2*pi*u2) for u2 in [0, 1) with an exact quadrant reduction."""
    u2 = np.asarray(u2, dtype=np.float64)
    v = 4.0 * u2
    quad = np.floor(v)
    f = v - quad
    hi = f > 0.5
    g = np.where(hi, 1.0 - f, f)
    c, s = _cos_sin_poly(_HALF_PI * g)
    # cos(pi/2 * f): f <= 1/2 -> cos(x); f > 1/2 -> sin(pi/2 (1-f)).
    cf = np.where(hi, s, c)
    sf = np.where(hi, c, s)  # sin(pi/2 * f)
    q = quad.astype(np.int64)
    return np.select([q == 0, q == 1, q == 2, q == 3], [cf, -sf, -cf, sf])


def words_to_uniforms(w0, w1):
    """u1 in (0, 1] from w0 and u2 in [0, 1) from w1, 53 bits each."""
    scale = 2.0 ** -53
    u1 = ((w0 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * scale
    u2 = (w1 >> np.uint64(11)).astype(np.float64) * scale
    return u1, u2


def box_muller(u1, u2):
    r = np.sqrt(-2.0 * series_ln(u1))
    return r * series_cos_2pi(u2)


def omega(n, ell, seed, sub=0, tag=TAG_OMEGA):
    """The n x ell standard Gaussian test matrix Psi (paper) / Omega, float64.

    Entry (i, j) comes from Philox4x64-10 at counter (i, j, tag, sub) with key
    (seed, 0).
    """
    i = np.arange(n, dtype=np.uint64)[:, None]
    j = np.arange(ell, dtype=np.uint64)[None, :]
    ctr = np.empty((n, ell, 4), dtype=np.uint64)
    ctr[..., 0] = i
    ctr[..., 1] = j
    ctr[..., 2] = np.uint64(tag)
    ctr[..., 3] = np.uint64(sub)
    key = np.array([np.uint64(seed & 0xFFFFFFFFFFFFFFFF), np.uint64(0)], dtype=np.uint64)
    w = philox4x64_10(ctr, key)
    u1, u2 = words_to_uniforms(w[..., 0], w[..., 1])
    return box_muller(u1, u2)
