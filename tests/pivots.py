"""Pivot comparison by margin (eq. 8): another implementation's QRCP pivots
against the oracle's arithmetic.

Two QRCPs that sum their column norms in different orders see norms that
differ by rounding, so where two trailing columns are nearly equal in norm
either choice is correct.  The rule: replay the other pivot sequence in the
oracle (``qrcp(follow=...)``) and, at every step s, compare the norm of the
column it chose with the largest norm the oracle sees at that step.  The
choice must be the oracle's (the first largest) unless the two norms are
within ``tau``; such near-tie steps are listed, not failed.

tau for identical input bits: Householder QR is column-wise backward stable,
the trailing columns of both computations are within c l u ||D_j|| of the
exact ones (u = 2^-53, small constant c), so their norms differ by at most
2 c l u max_j ||D_j||; the rule takes c = 4, tau = 8 l u max_j ||D_j||.
End to end, where the two cores themselves differ, ``extra`` adds the
perturbation bound of the path (||D_gpu - D_oracle||_2 <= ||D_gpu -
D_oracle||_F).
"""
import numpy as np

from oracle.dense import qrcp

U64 = 2.0 ** -53


def margin_tau(D, extra=0.0):
    D = np.asarray(D, dtype=np.float64)
    return 8.0 * D.shape[0] * U64 * float(np.max(np.linalg.norm(D, axis=0))) + float(extra)


def pivot_margins(D, piv, tau):
    """Returns the list of (step, gap) where piv's choice differs from the
    oracle's argmax; raises AssertionError at the first step whose gap
    exceeds tau (gap = sqrt(largest norm^2) - sqrt(chosen norm^2))."""
    piv = np.asarray(piv).astype(np.int64)
    trace = []
    qrcp(D, follow=piv, trace=trace)
    near = []
    for s, (acc, c) in enumerate(trace):
        j = int(np.argmax(acc))
        if j == c:
            continue
        gap = float(np.sqrt(acc[j]) - np.sqrt(acc[c]))
        assert gap <= tau, "step %d: chose position %d, largest %d, norm gap %.3e > tau %.3e" % (
            s, s + c, s + j, gap, tau)
        near.append((s, gap))
    return near
