"""GPU parity of the batched primality tests (paper Section 3.2: Alg. 2
modular powers, Alg. 3 Fermat, deterministic Miller-Rabin) against the CPU
oracle and against the sieve itself."""
import math
import os

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _rows(name):
    with open(os.path.join(GOLDEN, name)) as f:
        for line in f:
            line = line.split("#", 1)[0].strip()
            if line:
                yield [int(x) for x in line.split()]


@pytest.fixture(scope="module")
def gpu():
    import torch

    import paper_1205_4883_amd as sv

    assert torch.cuda.is_available()
    s = sv.Sieve(0)
    yield s
    s.close()


def test_small_n_equal_trial_division(gpu, oracle_mod):
    ns = np.arange(0, 20000, dtype=np.uint64)
    got = gpu.is_prime(ns)
    want = np.array([oracle_mod.trial_division_is_prime(int(n)) for n in ns])
    assert np.array_equal(got, want)


def test_equals_sieve_bitmap_near_1e12_and_1e15(gpu):
    for lo, hi in [(10**12 - 10**5, 10**12 + 10**5), (10**15 - 2 * 10**5, 10**15)]:
        words, _ = gpu.bitmap(lo, hi)
        bits = np.unpackbits(words.cpu().numpy().view(np.uint8), bitorder="little")
        nb = hi // 2 - lo // 2
        first = (lo & ~1) + 1
        odd = first + 2 * np.arange(nb, dtype=np.uint64)
        assert np.array_equal(gpu.is_prime(odd), bits[:nb].astype(bool))
        evens = odd + np.uint64(1)
        assert not gpu.is_prime(evens).any()


def test_queues_full_of_primes_and_of_pseudoprime_candidates(gpu, oracle_mod):
    # the kernel queues undecided candidates in LDS per chunk of 4096: a batch
    # of nothing but primes fills both queues, a batch of odd composites with
    # no factor up to 37 fills the first; ragged lengths leave partial chunks
    words, _ = oracle_mod.bitmap(10**15 - 6 * 10**5, 10**15)
    bits = np.unpackbits(words.view(np.uint8), bitorder="little")[: (6 * 10**5) // 2].astype(bool)
    odd = (10**15 - 6 * 10**5 + 1) + 2 * np.arange(bits.size, dtype=np.uint64)
    primes = odd[bits]
    assert primes.size > 4096 * 3
    for n in [primes.size, 4096 * 3 + 17, 4095, 1]:
        assert gpu.is_prime(primes[:n]).all()
    small = np.array([3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37], dtype=np.uint64)
    rough = odd[~bits]
    rough = rough[np.all(rough[:, None] % small[None, :] != 0, axis=1)]
    assert rough.size > 4096 * 2
    assert not gpu.is_prime(rough).any()
    mixed = np.concatenate([rough[:5000], primes[:5000]])
    np.random.default_rng(5).shuffle(mixed)
    got = gpu.is_prime(mixed)
    assert np.array_equal(got, np.isin(mixed, primes[:5000]))


def test_random_u64_equal_oracle_mr(gpu, oracle_mod):
    rng = np.random.default_rng(17)
    ns = rng.integers(0, 2**63, 40000, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    ns[:1000] = rng.integers(0, 2**40, 1000, dtype=np.uint64) | np.uint64(1)
    got = gpu.is_prime(ns)
    want = np.array([oracle_mod.mr_is_prime(int(n)) for n in ns])
    assert np.array_equal(got, want)
    assert got.sum() > 500  # about 1 in 22 odd 64-bit numbers is prime


def test_landmarks_thresholds_and_carmichael(gpu):
    vals, want = [], []
    for n, p in _rows("prime_landmarks.txt"):
        vals.append(n)
        want.append(bool(p))
    # the smallest strong pseudoprimes to the first k prime bases (each
    # sits exactly at a switch of the number of bases used)
    for n in [2047, 1373653, 25326001, 3215031751, 2152302898747, 3474749660383,
              341550071728321, 3825123056546413051]:
        vals.append(n)
        want.append(False)
    for (n,) in _rows("carmichael.txt"):
        vals.append(n)
        want.append(False)
    vals += [0, 1, 2, 3, 4, 2**64 - 1, 2**64 - 59, 2**61 - 1, 2**32 + 15]
    want += [False, False, True, True, False, False, True, True, True]
    assert list(gpu.is_prime(np.array(vals, dtype=np.uint64))) == want


def test_fermat_alg3_matches_oracle(gpu, oracle_mod):
    carm = [r[0] for r in _rows("carmichael.txt")]
    # bases 2, 7, 13 are prime to every listed Carmichael number except where
    # they divide it; draws d give base d + 1 for n > d + 1
    draws = [1, 6, 12]
    rng = np.random.default_rng(4)
    ns = np.concatenate([np.array(carm, dtype=np.uint64),
                         rng.integers(2, 10**12, 3000, dtype=np.uint64),
                         np.array([0, 1, 2, 3, 4, 6, 9, 15, 341, 561], dtype=np.uint64)])
    got = gpu.fermat(ns, draws)
    want = np.array([oracle_mod.fermat(int(n), draws) for n in ns])
    assert np.array_equal(got, want)
    for i, n in enumerate(carm):
        if all(math.gcd(d + 1, n) == 1 for d in draws):
            assert got[i], n  # fooled, as the paper warns
