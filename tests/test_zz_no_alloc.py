"""GPU tests of the allocation-free range call (sieve_range_bitmap_noalloc).

It must give exactly what sieve_range_bitmap gives (words and count) and
what the oracle gives, call after call, while keeping its counters in the
library's own per-GPU array.  Every comparison is exact.
"""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def env():
    import torch

    import paper_1205_4883_amd as sv

    assert torch.cuda.is_available()
    s = sv.Sieve(0)
    yield sv, torch, s
    s.close()


def _noalloc(sv, torch, s, lo, hi, bitmap=True):
    """One allocation-free call into outputs allocated beforehand (poisoned
    with -1, two spare words past the end): (words or None, pi)."""
    n = sv.sieve_bitmap_words(lo, hi)
    words = torch.full((n + 2,), -1, dtype=torch.int32, device="cuda:0") if bitmap else None
    d_pi = torch.full((1,), -1, dtype=torch.int64, device="cuda:0")
    stream = torch.cuda.current_stream(0)
    sv.sieve_range_bitmap_noalloc(s.ctx, lo, hi, words, n if bitmap else 0, d_pi, stream=stream)
    torch.cuda.synchronize()
    got = None
    if bitmap:
        w = words.cpu().numpy().view(np.uint32)
        assert np.all(w[n:] == 0xFFFFFFFF), "words past the range were written"
        got = w[:n]
    return got, int(d_pi.item())


def _plain(sv, torch, s, lo, hi):
    words, pi = s.bitmap(lo, hi)
    return words.cpu().numpy().view(np.uint32), pi


@pytest.mark.parametrize("cases", [
    # each pair runs back to back, the second call smaller than the first
    [(10**9 + 12345, 10**9 + 12345 + 40_000_003), (999_983, 1_000_000 + 70_001)],
    [(2, 10**9), (0, 100_003)],
    [(10**12 - 2 * 10**7 - 77, 10**12 - 7), (10**12 - 4099, 10**12 - 7)],
])
def test_noalloc_equals_plain_call_and_oracle_twice_in_a_row(env, oracle_mod, cases):
    sv, torch, s = env
    for lo, hi in cases:
        print(f"case noalloc bitmap [{lo}, {hi})", flush=True)
        got, pi = _noalloc(sv, torch, s, lo, hi)
        ref, ref_pi = _plain(sv, torch, s, lo, hi)
        assert pi == ref_pi, (lo, hi, pi, ref_pi)
        assert np.array_equal(got, ref), (lo, hi)
        want, want_pi = oracle_mod.bitmap(lo, hi)
        assert want_pi == pi and np.array_equal(got, want), (lo, hi)


def test_noalloc_count_only(env, oracle_mod):
    sv, torch, s = env
    for lo, hi, want in [(2, 10**10, 455052511), (2, 10**7, 664579), (10**11, 10**11 + 10**6, None)]:
        print(f"case noalloc count [{lo}, {hi})", flush=True)
        _, pi = _noalloc(sv, torch, s, lo, hi, bitmap=False)
        assert pi == sv.sieve_range_count(s.ctx, lo, hi)
        assert pi == (want if want is not None else oracle_mod.count(lo, hi))


@pytest.mark.parametrize("lo,hi,pi", [(5, 5, 0), (2, 3, 1), (0, 2, 0), (0, 3, 1), (3, 4, 1), (0, 0, 0)])
def test_noalloc_tiny_and_empty_ranges(env, lo, hi, pi):
    sv, torch, s = env
    print(f"case noalloc tiny [{lo}, {hi})", flush=True)
    got, got_pi = _noalloc(sv, torch, s, lo, hi)
    assert got_pi == pi
    ref, ref_pi = _plain(sv, torch, s, lo, hi)
    assert ref_pi == pi and np.array_equal(got, ref[: got.size])


def test_noalloc_needs_resident_base_primes(env, oracle_mod):
    sv, torch, s = env
    lo, hi = 3 * 10**12, 3 * 10**12 + 1_000_003  # isqrt(hi - 1) > 2^20
    if sv.sieve_plan(lo, hi)["sqrt_bound"] > 1 << 20:
        with pytest.raises(sv.SieveError) as e:
            _noalloc(sv, torch, s, lo, hi)
        assert e.value.status == -2  # SIEVE_ERANGE, nothing queued
    s.base_primes(1_800_000)  # grow the table outside the allocation-free call
    print(f"case noalloc bitmap [{lo}, {hi}) after growing the base primes", flush=True)
    got, pi = _noalloc(sv, torch, s, lo, hi)
    ref, ref_pi = _plain(sv, torch, s, lo, hi)
    assert pi == ref_pi and np.array_equal(got, ref)
    want, want_pi = oracle_mod.bitmap(lo, hi)
    assert want_pi == pi and np.array_equal(got, want)


def test_noalloc_argument_errors(env):
    sv, torch, s = env
    d_pi = torch.zeros(1, dtype=torch.int64, device="cuda:0")
    words = torch.zeros(4, dtype=torch.int32, device="cuda:0")
    for args, status in [((10, 5, words, 4, d_pi), -1), ((0, 10**15 + 1, None, 0, d_pi), -2),
                         ((0, 1000, words, 4, d_pi), -4)]:
        with pytest.raises(sv.SieveError) as e:
            sv.sieve_range_bitmap_noalloc(s.ctx, *args)
        assert e.value.status == status
    with pytest.raises(sv.SieveError):
        sv.sieve_range_bitmap_noalloc(None, 0, 10, None, 0, d_pi)
