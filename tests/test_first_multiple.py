"""CPU check of the segment kernels' start computation (first_multiple in
sieve_kernels.hip), replayed step by step in numpy float64.

For a segment whose bit 0 is the odd integer n0 and a base prime p, the
kernels need the first odd multiplier m0 >= p with m0 * p >= n0 (crossing off
starts at max(p^2, n0), Section 3.1), as the bit offset (m0 * p - n0) / 2 and
m0 mod 30.  They take floor(n0 * (1/p)) in double, where 1/p is rounded to
double once per prime, get the remainder with one fused multiply-add, and
correct the quotient once.  The exact answer here comes from Python integers.
The inputs include multiples of p and their neighbours near 10^15 and 2^50,
and the multiples on which the double quotient is one too small.

numpy's float64 multiply, floor and division round as the device's v_mul_f64,
v_floor_f64 and IEEE division do.  numpy has no fused multiply-add, but both
remainders the kernel forms, n0 - q*p and q - 30*t, are integers below 2^53
in magnitude, which a fused multiply-add returns exactly; they are formed in
int64 here.
"""
from fractions import Fraction

import numpy as np
import pytest

LIM = 1 << 28  # the offset cap the carried-start path passes


def replay(n0, p, lim_bits=LIM, correct=True):
    """first_multiple's steps on arrays n0 (odd, int64) and p (int64)."""
    nf = n0.astype(np.float64)
    pf = p.astype(np.float64)
    inv = np.float64(1.0) / pf
    q = np.floor(nf * inv).astype(np.int64)
    r = n0 - q * p  # the fma: exact
    if correct:
        neg = r < 0
        r = np.where(neg, r + p, r)
        q = np.where(neg, q - 1, q)
        big = r >= p
        r = np.where(big, r - p, r)
        q = np.where(big, q + 1, q)
    d = np.where(r > 0, p - r, 0)
    q = np.where(r > 0, q + 1, q)
    t = np.floor(q.astype(np.float64) * (np.float64(1.0) / np.float64(30.0))).astype(np.int64)
    k30 = q - 30 * t  # the second fma: exact
    k30 = np.where(k30 < 0, k30 + 30, k30)
    k30 = np.where(k30 >= 30, k30 - 30, k30)
    even = (k30 & 1) == 0
    d = np.where(even, d + p, d)
    k30 = np.where(even, k30 + 1, k30)
    off = d >> 1
    m30 = k30
    past = pf * pf > nf
    o2 = (p * p - n0) >> 1
    off = np.where(past, np.minimum(o2, lim_bits), off)
    m30 = np.where(past, p % 30, m30)
    return off, m30


def exact(n0, p, lim_bits=LIM):
    offs, m30s = [], []
    for a, b in zip(n0.tolist(), p.tolist()):
        k = max(-(-a // b), b)
        if k % 2 == 0:
            k += 1
        offs.append(min((k * b - a) // 2, lim_bits) if k == b else (k * b - a) // 2)
        m30s.append(k % 30)
    return np.array(offs, dtype=np.int64), np.array(m30s, dtype=np.int64)


# primes near 37, 2^16, 2^20, 2^24 and the largest base prime of the domain
PRIMES = [37, 41, 65521, 65537, 1048573, 1048583, 16777213, 16777259, 31622743, 31622777]


def _inputs(centres, rng, per=400):
    n0, p = [], []
    for q in PRIMES:
        for c in centres:
            ks = c // q + rng.integers(-per, per, per)
            for d in (-2, -1, 0, 1, 2):
                n = ks * q + d
                n = n[(n % 2 == 1) & (n > 0)]
                n0.append(n)
                p.append(np.full(n.size, q, dtype=np.int64))
    return np.concatenate(n0).astype(np.int64), np.concatenate(p)


@pytest.mark.parametrize("centres", [[10**15 - 2 * 10**9], [1 << 50], [10**12, 3 * 10**13], [10**6, 10**9]])
def test_start_is_exact_on_multiples_and_their_neighbours(centres):
    rng = np.random.default_rng(7)
    n0, p = _inputs(centres, rng)
    off, m30 = replay(n0, p)
    want_off, want_m30 = exact(n0, p)
    assert np.array_equal(off, want_off)
    assert np.array_equal(m30, want_m30)


def test_start_at_the_square_of_the_prime():
    # segments that begin below p^2: crossing off starts at p^2 (m0 = p)
    p = np.array(PRIMES, dtype=np.int64)
    for d in (-4, -2, 0, 2):
        n0 = p * p + d
        n0 = np.where(n0 % 2 == 0, n0 - 1, n0)
        off, m30 = replay(n0, p)
        want_off, want_m30 = exact(n0, p)
        assert np.array_equal(off, want_off) and np.array_equal(m30, want_m30)


def _is_prime(n):
    return n > 1 and all(n % d for d in range(2, int(n ** 0.5) + 1))


def _adversarial():
    """Odd n0 = k*p with k just below a power of two, for primes p whose
    double reciprocal is rounded down by more than 2^-54 relative: there the
    double product n0 * (1/p) can round to just below k, and its floor is
    then k - 1.  (Below 2^53 no other n0 can move the floor: n0 / p is at
    least 1/p away from the next integer otherwise.)"""
    n0, p = [], []
    for base in (37, 1000, 65521, 1048573, 16777213, 31622700):
        q, found = base, 0
        while found < 12:
            if _is_prime(q):
                found += 1
                if Fraction(1.0 / q) * q - 1 < -Fraction(1, 1 << 54):
                    for m in range(8, 53):
                        for j in (1, 2, 3, 4):
                            k = (1 << m) - j
                            if k * q <= 10**15 and (k * q) % 2 == 1:
                                for d in (-2, 0, 2):
                                    n0.append(k * q + d)
                                    p.append(q)
            q += 1
    return np.array(n0, dtype=np.int64), np.array(p, dtype=np.int64)


def test_start_is_exact_where_the_double_quotient_is_off():
    n0, p = _adversarial()
    assert n0.size > 500
    off, m30 = replay(n0, p)
    want_off, want_m30 = exact(n0, p)
    assert np.array_equal(off, want_off)
    assert np.array_equal(m30, want_m30)


def test_the_raw_double_quotient_is_off_on_these_inputs():
    # floor(n0 * (1/p)) in double is one below floor(n0 / p) on some of these
    # inputs and never further off: the start is exact above only because
    # the steps after the product handle that case.  (Below 2^52, the only
    # case: n0 an exact multiple, remainder p, which the ceiling step takes
    # to an offset of 0; the explicit correction also covers the opposite
    # direction, which this domain never reaches.)
    n0, p = _adversarial()
    q = np.floor(n0.astype(np.float64) * (np.float64(1.0) / p.astype(np.float64))).astype(np.int64)
    err = q - n0 // p
    assert err.min() >= -1 and err.max() <= 0 and np.any(err != 0)
    rng = np.random.default_rng(11)
    n0, p = _inputs([10**15 - 2 * 10**9, 1 << 49], rng, per=50)
    q = np.floor(n0.astype(np.float64) * (np.float64(1.0) / p.astype(np.float64))).astype(np.int64)
    err = q - n0 // p
    assert err.min() >= -1 and err.max() <= 0
    off, m30 = replay(n0, p, correct=False)
    assert np.array_equal(off, exact(n0, p)[0])
