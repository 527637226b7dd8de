"""Index division used by every grid kernel (mbx_dev.h divmod): the quotient
of n by an extent d is the truncated FP64 product n * inv with inv the
smallest double >= 1/d (set up on the host), exact with no correction step
for 0 <= n < 2^31, 1 <= d <= 2^21 and n/d < 2^24.  The device computes the
same IEEE operations as below: a correctly rounded multiply and a truncating
conversion.  Checked here on the divisors and numerators where it could fail:
exact multiples of d, one below them and the top of each remainder range."""
from fractions import Fraction

import numpy as np

NMAX = 2 ** 31 - 1


def rcp_up(d):
    r = 1.0 / d
    if Fraction(r) * d < 1:
        r = float(np.nextafter(r, 2.0))
    return r


def _numerators(d, rng):
    top = min(NMAX // d, 2 ** 24 - 1)
    qs = np.unique(np.concatenate([np.arange(0, 32), rng.integers(0, top + 1, 64), [top]])).astype(np.int64)
    n = np.concatenate([qs * d, qs * d - 1, qs * d + d - 1])
    return n[(n >= 0) & (n <= NMAX) & (n // d < 2 ** 24)]


def _divisors(rng):
    return sorted(set(range(1, 1025)) | {2 ** k for k in range(22)} | {2 ** k - 1 for k in range(1, 22)}
                  | {int(v) for v in rng.integers(1025, 2 ** 21 + 1, 400)})


def test_round_up_reciprocal_gives_exact_quotients():
    rng = np.random.default_rng(11)
    for d in _divisors(rng):
        inv = rcp_up(d)
        assert Fraction(inv) >= Fraction(1, d) and Fraction(inv) * d - 1 < Fraction(1, 2 ** 51)
        n = _numerators(d, rng)
        q = np.trunc(n.astype(np.float64) * inv).astype(np.int64)
        np.testing.assert_array_equal(q, n // d, err_msg=f"d = {d}")
        r = n - q * d
        assert np.all((r >= 0) & (r < d))


def test_round_to_nearest_reciprocal_needs_a_correction():
    # with RN(1/d) below 1/d the truncated product falls one short at exact
    # multiples for some divisors: the reason the host rounds the reciprocal up
    rng = np.random.default_rng(12)
    short = 0
    for d in _divisors(rng):
        n = _numerators(d, rng)
        q = np.trunc(n.astype(np.float64) * (1.0 / d)).astype(np.int64)
        short += int(np.sum(q != n // d))
    assert short > 0
