"""Pins for the oracle's Gaussian test-matrix stream (Sec. 3.1, Algorithm 1 first step).

Against things other than the oracle itself:
* numpy's independent Philox4x64-10 bit generator (which bumps its counter
  once before producing its first block);
* libm's log / cos / sqrt within a few ulp;
* distributional checks (moments, Kolmogorov-Smirnov) for "i.i.d. standard
  Gaussian".
"""
import numpy as np
import pytest
from scipy import stats

from oracle import philox as P

U64 = 0xFFFFFFFFFFFFFFFF


def _numpy_block(counter, key):
    # numpy increments the 256-bit counter (word 0 least significant) before
    # generating; undo that with a full borrow chain.
    v = sum(int(w) << (64 * i) for i, w in enumerate(counter))
    v = (v - 1) % (1 << 256)
    c = [(v >> (64 * i)) & U64 for i in range(4)]
    bg = np.random.Philox(counter=np.array(c, dtype=np.uint64),
                          key=np.array([int(x) for x in key], dtype=np.uint64))
    return [int(x) for x in bg.random_raw(4)]


@pytest.mark.parametrize("counter,key", [
    ((0, 0, 0, 0), (0, 0)),
    ((5, 6, 7, 8), (1, 2)),
    ((U64, U64, U64, U64), (U64, U64)),
    ((123456789, 0, 0, 17), (0xDEADBEEFCAFEF00D, 0)),
    ((1, 2**63, 3, 2**40), (7, 9)),
])
def test_philox_matches_numpy(counter, key):
    ours = [int(x) for x in P.philox4x64_10(list(counter), list(key))]
    assert ours == _numpy_block(counter, key)


def test_philox_vectorised_equals_scalar():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**63, size=(64, 4), dtype=np.uint64)
    key = np.array([42, 0], dtype=np.uint64)
    vec = P.philox4x64_10(ctr, key)
    for i in range(0, 64, 7):
        assert [int(x) for x in vec[i]] == [int(x) for x in P.philox4x64_10(ctr[i], key)]
        assert [int(x) for x in vec[i]] == _numpy_block([int(x) for x in ctr[i]], [42, 0])


def _ulp_err(a, b):
    return np.abs(a - b) / np.spacing(np.abs(b))


def test_series_ln_close_to_libm():
    rng = np.random.default_rng(1)
    a = rng.integers(1, 2**53 + 1, size=200000, dtype=np.uint64)
    u = a.astype(np.float64) * 2.0 ** -53
    u = np.concatenate([u, [2.0 ** -53, 0.5, 1.0, np.sqrt(0.5), np.nextafter(np.sqrt(2) / 2, 1)]])
    ours = P.series_ln(u)
    ref = np.log(u)
    nz = ref != 0
    assert np.max(_ulp_err(ours[nz], ref[nz])) <= 4.0
    assert ours[u == 1.0][0] == 0.0


def test_series_cos_close_to_libm():
    rng = np.random.default_rng(2)
    b = rng.integers(0, 2**53, size=200000, dtype=np.uint64)
    u = b.astype(np.float64) * 2.0 ** -53
    u = np.concatenate([u, [0.0, 0.125, 0.25, 0.5, 0.75, 0.375, 1 - 2.0 ** -53]])
    ours = P.series_cos_2pi(u)
    ref = np.cos(2.0 * np.pi * u)
    # |error| bound: a few ulp of 1 (the reference itself rounds 2*pi*u).
    assert np.max(np.abs(ours - ref)) <= 4e-16 + 4 * np.pi * 2.0 ** -53
    assert ours[-7] == 1.0
    assert ours[-4] == -1.0  # u2 = 1/2
    assert ours[-5] == 0.0   # u2 = 1/4 (exact zero from the reduction)


def test_box_muller_close_to_libm_and_exact_endpoints():
    w = P.philox4x64_10(np.stack([np.arange(50000, dtype=np.uint64)] + [np.zeros(50000, np.uint64)] * 3, -1),
                        np.array([9, 0], dtype=np.uint64))
    u1, u2 = P.words_to_uniforms(w[:, 0], w[:, 1])
    assert np.all(u1 > 0) and np.all(u1 <= 1) and np.all(u2 >= 0) and np.all(u2 < 1)
    z = P.box_muller(u1, u2)
    ref = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)
    radius = np.sqrt(-2.0 * np.log(u1))
    # absolute error relative to the radius: near a zero of cos the libm
    # reference's own rounding of 2*pi*u2 dominates any relative measure.
    assert np.max(np.abs(z - ref) / np.maximum(radius, 1.0)) < 4e-15
    # u1 = 1 gives radius exactly 0.
    assert P.box_muller(np.array([1.0]), np.array([0.3]))[0] == 0.0


def test_omega_is_standard_gaussian():
    Om = P.omega(4000, 250, seed=2024)
    x = Om.ravel()
    n = x.size
    assert abs(x.mean()) < 5.0 / np.sqrt(n)
    assert abs(x.var() - 1.0) < 5.0 * np.sqrt(2.0 / n)
    assert abs(stats.skew(x)) < 5.0 * np.sqrt(6.0 / n)
    assert abs(stats.kurtosis(x)) < 5.0 * np.sqrt(24.0 / n)
    assert stats.kstest(x, "norm").pvalue > 1e-4
    # columns are uncorrelated
    C = np.corrcoef(Om[:, :20].T)
    assert np.max(np.abs(C - np.eye(20))) < 6.0 / np.sqrt(4000)


def test_omega_layout_nested_and_seeded():
    a = P.omega(300, 12, seed=5)
    b = P.omega(500, 20, seed=5)
    np.testing.assert_array_equal(a, b[:300, :12])
    c = P.omega(300, 12, seed=6)
    d = P.omega(300, 12, seed=5, sub=1)
    assert not np.any(a == c) or np.mean(a == c) < 1e-3
    assert np.mean(a == d) < 1e-3
    # entry (i, j) is the Box-Muller of the Philox block at counter (i, j, 0, sub)
    w = P.philox4x64_10([7, 3, 0, 0], [5, 0])
    u1, u2 = P.words_to_uniforms(np.array([w[0]]), np.array([w[1]]))
    assert P.box_muller(u1, u2)[0] == a[7, 3]
