"""Pins of the CPU oracle against facts fixed outside it (CPU only).

Each test ties an oracle function to something the oracle did not compute:
published values (tests/golden/, each file names its source), brute force on
small inputs, closed forms, or invariants that any correct sieve satisfies.
The oracle follows the paper's definition of the result (Sections 1 and 3.1)
and its auxiliary algorithms (Section 3.2, Algs. 2 and 3).
"""
import math
import os
import random

import numpy as np
import pytest

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield [int(x) for x in line.split()]


def _bits(words, nbits):
    """Unpack LSB-first uint32 words into a 0/1 array of nbits entries."""
    b = np.unpackbits(np.asarray(words, dtype="<u4").view(np.uint8), bitorder="little")
    return b[:nbits]


def _brute_bitmap(lo, hi):
    """Odd-only bitmap of [lo, hi) by trial division of each odd integer,
    plus pi.  Written independently of the oracle's sieve, in Python."""
    first = (lo & ~1) + 1
    nbits = hi // 2 - lo // 2
    bits = []
    for i in range(nbits):
        n = first + 2 * i
        bits.append(1 if n >= 2 and all(n % d for d in range(2, math.isqrt(n) + 1)) else 0)
    pi = sum(bits) + (1 if lo <= 2 < hi else 0)
    return bits, pi


# -- isqrt ---------------------------------------------------------------

def test_isqrt_matches_python(oracle_mod):
    rng = random.Random(1)
    vals = [0, 1, 2, 3, 4, 15, 16, 17, 2**32 - 1, 2**32, 2**64 - 1, 10**15, 10**15 - 1]
    for r in [1, 2, 3, 1000, 31622776, 2**32 - 1]:
        vals += [r * r - 1, r * r, r * r + 1]
    vals += [rng.randrange(2**64) for _ in range(2000)]
    for n in vals:
        if n < 2**64:
            assert oracle_mod.isqrt(n) == math.isqrt(n), n


# -- trial division and Miller-Rabin ------------------------------------

def test_trial_division_small_primes_by_definition(oracle_mod):
    # primes below 100, written out
    known = [2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37, 41, 43, 47, 53, 59, 61,
             67, 71, 73, 79, 83, 89, 97]
    got = [n for n in range(100) if oracle_mod.trial_division_is_prime(n)]
    assert got == known


def test_mr_equals_trial_division_below_2e5(oracle_mod):
    for n in range(200_000):
        assert oracle_mod.mr_is_prime(n) == oracle_mod.trial_division_is_prime(n), n


@pytest.mark.parametrize("n,is_prime", list(_rows("prime_landmarks.txt")))
def test_mr_landmarks(oracle_mod, n, is_prime):
    assert oracle_mod.mr_is_prime(n) == bool(is_prime)


def test_mr_random_products_are_composite(oracle_mod):
    rng = random.Random(2)
    primes = [p for p in range(3, 5000) if oracle_mod.trial_division_is_prime(p)]
    for _ in range(2000):
        a, b = rng.choice(primes), rng.choice(primes)
        c = rng.choice(primes)
        assert not oracle_mod.mr_is_prime(a * b)
        assert not oracle_mod.mr_is_prime(a * b * c)


# -- Alg. 2 and Alg. 3 (Section 3.2) -------------------------------------

def test_modpow_matches_python_pow(oracle_mod):
    rng = random.Random(3)
    for _ in range(5000):
        a = rng.randrange(2**64)
        b = rng.randrange(2**64)
        c = rng.randrange(1, 2**64)
        assert oracle_mod.modpow(a, b, c) == pow(a, b, c)
    # edge cases: b = 0 gives 1 mod c; c = 1 gives 0
    assert oracle_mod.modpow(5, 0, 7) == 1
    assert oracle_mod.modpow(5, 0, 1) == 0
    assert oracle_mod.modpow(0, 5, 7) == 0
    assert oracle_mod.modpow(2, 10, 1000) == 24


def test_fermat_little_theorem_on_primes(oracle_mod):
    # Eq. 6: a^(p-1) = 1 (mod p) for prime p and 0 < a < p
    for p in [3, 5, 7, 97, 7919, 2147483647, 999999999989, 18446744073709551557]:
        for a in [1, 2, 3, p - 1]:
            if 0 < a < p:
                assert oracle_mod.modpow(a, p - 1, p) == 1


def test_fermat_fooled_by_carmichael_but_not_sieve(oracle_mod):
    carm = [r[0] for r in _rows("carmichael.txt")]
    for n in carm:
        # coprime bases pass Alg. 3 although n is composite
        draws = [a - 1 for a in range(2, 60) if math.gcd(a, n) == 1]
        assert oracle_mod.fermat(n, draws)
        assert not oracle_mod.mr_is_prime(n)
        assert not oracle_mod.trial_division_is_prime(n)
        # the sieve clears the Carmichael number's bit
        lo, hi = n - 10, n + 10
        words, _ = oracle_mod.bitmap(lo, hi)
        first = (lo & ~1) + 1
        assert _bits(words, hi // 2 - lo // 2)[(n - first) // 2] == 0
    # Alg. 3 rejects p = 1 and an obvious composite with a non-witness-free base
    assert not oracle_mod.fermat(1, [0])
    assert not oracle_mod.fermat(15, [1])  # base 2: 2^14 mod 15 = 4


# -- the sieve: definition, brute force, published counts -----------------

def test_sieve_primes_below_1e5_equal_trial_division(oracle_mod):
    hi = 100_001
    words, pi = oracle_mod.bitmap(0, hi)
    bits = _bits(words, hi // 2)
    for i in range(hi // 2):
        n = 2 * i + 1
        assert bits[i] == int(oracle_mod.trial_division_is_prime(n)), n
    assert pi == sum(oracle_mod.trial_division_is_prime(n) for n in range(hi))


def test_sieve_every_tiny_range(oracle_mod):
    # every (lo, hi) with 0 <= lo <= hi <= 160 against Python trial division
    ref = {}
    for lo in range(0, 161):
        for hi in range(lo, 161):
            words, pi = oracle_mod.bitmap(lo, hi)
            bits, rpi = _brute_bitmap(lo, hi)
            nbits = hi // 2 - lo // 2
            assert list(_bits(words, nbits)) == bits, (lo, hi)
            assert pi == rpi, (lo, hi)
            assert oracle_mod.count(lo, hi) == rpi
            ref[(lo, hi)] = rpi
    assert ref[(0, 160)] == 37


def test_sieve_random_small_ranges(oracle_mod):
    rng = random.Random(4)
    for _ in range(300):
        lo = rng.randrange(0, 20000)
        hi = lo + rng.randrange(0, 3000)
        words, pi = oracle_mod.bitmap(lo, hi)
        bits, rpi = _brute_bitmap(lo, hi)
        assert list(_bits(words, hi // 2 - lo // 2)) == bits, (lo, hi)
        assert pi == rpi


@pytest.mark.parametrize("k,pi", [r for r in _rows("pi_powers_of_ten.txt") if r[0] <= 10])
def test_sieve_pi_powers_of_ten(oracle_mod, k, pi):
    assert oracle_mod.count(0, 10**k) == pi
    assert oracle_mod.count(2, 10**k) == pi
    assert oracle_mod.count(0, 10**k + 1) == pi  # 10^k is composite


@pytest.mark.parametrize("lo,hi,pi", list(_rows("pi_landmarks.txt")))
def test_sieve_pi_landmarks(oracle_mod, lo, hi, pi):
    assert oracle_mod.count(lo, hi) == pi


def test_sieve_single_thread_equals_threaded(oracle_mod):
    for lo, hi in [(0, 10**8), (123456789, 123456789 + 7 * 2**21 + 99)]:
        assert oracle_mod.count(lo, hi, threads=1) == oracle_mod.count(lo, hi, threads=8)
        w1, p1 = oracle_mod.bitmap(lo, hi, threads=1)
        w8, p8 = oracle_mod.bitmap(lo, hi, threads=8)
        assert p1 == p8 and np.array_equal(w1, w8)


def test_sieve_near_1e12_against_miller_rabin(oracle_mod):
    # bits around the landmarks, each decided independently by Miller-Rabin
    for lo, hi in [(10**12 - 2000, 10**12 + 2000), (999999999989, 999999999990),
                   (999999999990, 1000000000039), (999999999990, 1000000000040)]:
        words, pi = oracle_mod.bitmap(lo, hi)
        nbits = hi // 2 - lo // 2
        bits = _bits(words, nbits)
        first = (lo & ~1) + 1
        mr = [int(oracle_mod.mr_is_prime(first + 2 * i)) for i in range(nbits)]
        assert list(bits) == mr
        assert pi == sum(mr)
    assert oracle_mod.count(999999999990, 1000000000039) == 0
    assert oracle_mod.count(999999999990, 1000000000040) == 1
    assert oracle_mod.count(999999999989, 999999999990) == 1


def test_sieve_block_boundaries_against_miller_rabin(oracle_mod):
    # ranges that straddle the oracle's internal 2^20-odd-integer blocks
    rng = random.Random(5)
    for base in [2**21, 3 * 2**21, 10**11]:
        for d in [-130, -65, -64, -63, -1, 0, 1, 63, 64, 65]:
            lo = base + d
            hi = lo + 2**21 + 777
            words, pi = oracle_mod.bitmap(lo, hi)
            nbits = hi // 2 - lo // 2
            bits = _bits(words, nbits)
            first = (lo & ~1) + 1
            for i in [0, 1, nbits - 1, nbits - 2] + [rng.randrange(nbits) for _ in range(300)]:
                assert bits[i] == oracle_mod.mr_is_prime(first + 2 * i), (lo, hi, i)
            assert pi == int(bits.sum()) + (1 if lo <= 2 < hi else 0)


def test_sieve_base_prime_square_edges(oracle_mod):
    # hi = p^2 excludes p^2; hi = p^2 + 1 includes it, and it must be composite
    for p in [3, 5, 7, 11, 13, 31, 37, 1009, 31607]:
        sq = p * p
        assert oracle_mod.count(sq - 1, sq) == int(oracle_mod.mr_is_prime(sq - 1))
        assert oracle_mod.count(sq, sq + 1) == 0
        words, _ = oracle_mod.bitmap(sq - 4, sq + 2)
        bits = _bits(words, (sq + 2) // 2 - (sq - 4) // 2)
        first = ((sq - 4) & ~1) + 1
        assert bits[(sq - first) // 2] == 0


def test_sieve_additivity(oracle_mod):
    rng = random.Random(6)
    for _ in range(40):
        a = rng.randrange(0, 10**11)
        c = a + rng.randrange(0, 10**7)
        b = rng.randrange(a, c + 1)
        assert oracle_mod.count(a, c) == oracle_mod.count(a, b) + oracle_mod.count(b, c)


def test_sieve_bitmap_concatenation(oracle_mod):
    # when b - a is a multiple of 64 (and a even), the words of [a, b) and
    # [b, c) concatenate to the words of [a, c)
    rng = random.Random(7)
    for _ in range(20):
        a = rng.randrange(0, 10**10) & ~1
        b = a + 64 * rng.randrange(0, 50000)
        c = b + rng.randrange(0, 3_000_000)
        wac, _ = oracle_mod.bitmap(a, c)
        wab, _ = oracle_mod.bitmap(a, b)
        wbc, _ = oracle_mod.bitmap(b, c)
        assert np.array_equal(wac, np.concatenate([wab, wbc]).astype(np.uint32))


def test_sieve_count_is_popcount_plus_two(oracle_mod):
    for lo, hi in [(0, 10**6), (1, 10**6), (2, 10**6), (3, 10**6), (10**9, 10**9 + 10**6)]:
        words, pi = oracle_mod.bitmap(lo, hi)
        pop = int(_bits(words, hi // 2 - lo // 2).sum())
        assert pi == pop + (1 if lo <= 2 < hi else 0)
        # pad bits of the last word are zero
        nbits = hi // 2 - lo // 2
        if nbits % 32:
            assert int(words[-1]) >> (nbits % 32) == 0


def test_sieve_errors_and_empty(oracle_mod):
    assert oracle_mod.status_of(5, 4, words=False) == oracle_mod.EINVAL
    assert oracle_mod.status_of(0, 10**15 + 1, words=False) == oracle_mod.ERANGE
    assert oracle_mod.status_of(0, 1000, n_words=15) == oracle_mod.EBUFSZ
    assert oracle_mod.status_of(0, 1000, n_words=16) == oracle_mod.OK
    for x in [0, 1, 2, 3, 10**12]:
        assert oracle_mod.count(x, x) == 0
    assert oracle_mod.count(0, 3) == 1  # {2}
    assert oracle_mod.count(2, 3) == 1
    assert oracle_mod.count(3, 4) == 1
    assert oracle_mod.count(0, 2) == 0


def test_base_primes(oracle_mod):
    p = oracle_mod.base_primes(100_000)
    assert len(p) == 9592 and p[0] == 2 and p[-1] == 99991
    assert len(oracle_mod.base_primes(31622)) == 3401
    assert len(oracle_mod.base_primes(3162)) == 446
    assert len(oracle_mod.base_primes(1)) == 0
    assert list(oracle_mod.base_primes(2)) == [2]
    assert all(oracle_mod.trial_division_is_prime(int(x)) for x in oracle_mod.base_primes(5000))
