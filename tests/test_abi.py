"""CPU tests of the C ABI: the library loads, exports what include/sieve.h
declares, and its pure host functions (planning, sizes, argument checks)
behave as documented.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    text = open(os.path.join(ROOT, "include", "sieve.h")).read()
    return sorted(set(re.findall(r"SIEVE_API\s+[\w\s\*]*?\b(sieve_\w+)\s*\(", text)))


def test_header_declares_the_boundary():
    names = _declared()
    for must in ["sieve_base_primes", "sieve_range_bitmap", "sieve_range_count", "sieve_batch"]:
        assert must in names


def test_library_exports_every_declared_symbol():
    import paper_1205_4883_amd as sv

    lib = ctypes.CDLL(sv.LIB_PATH)
    for name in _declared():
        assert hasattr(lib, name), name
    assert sorted(sv.EXPORTED) == _declared()


def test_bitmap_words():
    import paper_1205_4883_amd as sv

    assert sv.sieve_bitmap_words(2, 10**7) == 156250
    assert sv.sieve_bitmap_words(2, 10**9) == 15625000
    assert sv.sieve_bitmap_words(0, 0) == 0
    assert sv.sieve_bitmap_words(5, 4) == 0
    assert sv.sieve_bitmap_words(0, 64) == 1
    assert sv.sieve_bitmap_words(0, 65) == 1  # odd 1..63
    assert sv.sieve_bitmap_words(0, 66) == 2  # 65 opens a second word
    assert sv.sieve_bitmap_words(3, 4) == 1


def test_plan_sizes():
    import paper_1205_4883_amd as sv

    p = sv.sieve_plan(2, 10**10)
    assert p["nbits"] == 4999999999 and p["n_words"] == 156250000
    assert p["sqrt_bound"] == 99999
    assert p["n_segments"] * p["seg_bits"] >= p["nbits"]
    p = sv.sieve_plan(2, 10**9)
    assert p["sqrt_bound"] == 31622 and p["n_words"] == 15625000
    p = sv.sieve_plan(0, 122)
    assert p["sqrt_bound"] == 11
    p = sv.sieve_plan(0, 121)
    assert p["sqrt_bound"] == 10
    p = sv.sieve_plan(0, 0)
    assert p["nbits"] == 0 and p["n_segments"] == 0
    p = sv.sieve_plan(0, 10**15)
    assert p["sqrt_bound"] == 31622776


def test_plan_tuning_resolution():
    import paper_1205_4883_amd as sv

    p = sv.sieve_plan(2, 10**10, tuning=dict(seg_bits=65536, dense_limit=500, block_threads=512))
    assert p["seg_bits"] == 65536 and p["dense_limit"] == 500 and p["block_threads"] == 512
    p = sv.sieve_plan(2, 10**10, tuning=dict(dense_limit=3))
    assert p["dense_limit"] == 37
    # defaults: 2^19-bit segments with 1024 threads once a range fills the
    # chip; the widest segment (622,592 bits, still two workgroups per CU)
    # from four rounds of 2^19-bit segments (8 per CU) when no hit buckets
    # are wanted; smaller segments take fewer threads
    p = sv.sieve_plan(2, 10**10)
    assert p["seg_bits"] == 622592 and p["block_threads"] == 1024 and p["dense_limit"] == 1216
    # 954 segments of 2^19 bits are two rounds of 512 workgroups, the second
    # 86% full: the smallest segment that still needs two rounds fills both
    p = sv.sieve_plan(2, 10**9)
    assert p["seg_bits"] == 15360 * 32 and p["n_segments"] == 1018 and p["block_threads"] == 1024
    assert p["dense_limit"] == 960
    assert sv.sieve_plan(0, 2 * 2048 * 2**19)["seg_bits"] == 622592         # exactly 2048 segments
    q = sv.sieve_plan(0, 2 * 2047 * 2**19)                                  # 2047: four rounds, full
    assert q["seg_bits"] == 1 << 19 and q["n_segments"] == 2047
    q = sv.sieve_plan(0, 2 * 1025 * 2**19)                                  # 1025: three rounds
    assert q["n_segments"] <= 3 * 512 and q["seg_bits"] < 1 << 19 and q["seg_bits"] % 4096 == 0
    assert q["n_segments"] * q["seg_bits"] >= q["nbits"] and q["block_threads"] == 1024
    q = sv.sieve_plan(0, 2 * 513 * 2**19)                                   # 513: two rounds of about half
    assert q["n_segments"] <= 1024 and q["seg_bits"] <= (1 << 18) + 4096 and q["block_threads"] == 1024
    assert sv.sieve_plan(0, 2 * 512 * 2**19)["seg_bits"] == 1 << 19        # one full round stays
    assert sv.sieve_plan(2, 10**10, n_cu=64)["seg_bits"] == 622592
    # a device with 64 KiB of LDS per workgroup holds 2^18-bit segments at most
    assert sv.sieve_plan(2, 10**10, lds_bytes=65536)["seg_bits"] == 1 << 18
    p = sv.sieve_plan(2, 10**10, tuning=dict(seg_bits=1 << 18))
    assert p["block_threads"] == 512
    p = sv.sieve_plan(2, 10**10, tuning=dict(seg_bits=1 << 15))
    assert p["block_threads"] == 512
    p = sv.sieve_plan(2, 10**10, tuning=dict(seg_bits=1 << 13))
    assert p["block_threads"] == 256 and p["dense_limit"] == 128
    assert sv.sieve_plan(2, 10**7)["dense_limit"] == 128
    # hit buckets: automatic once sqrt(hi) reaches two segments (622592 bits
    # for the widest segment, which long ranges take: hi >= about 1.55e12) on
    # a range of at least 2^30 odd integers
    for lo in (2 * 10**12, 3 * 10**12):
        p = sv.sieve_plan(lo, lo + 10**10)
        assert p["bucket_limit"] == 622592 and p["seg_bits"] == 622592
    for lo in (10**11, 10**12):
        p = sv.sieve_plan(lo, lo + 10**10)
        assert p["bucket_limit"] == 0 and p["seg_bits"] == 622592
    edge = 1245184 ** 2  # sqrt(hi) = two widest segments exactly
    assert sv.sieve_plan(edge - 2**32, edge)["bucket_limit"] == 0
    assert sv.sieve_plan(edge - 2**32, edge + 2**22)["bucket_limit"] == 622592
    # 2^30 odd integers (the least that buckets take) are four rounds of
    # 2^19-bit segments on 256 CUs, so a bucketed range always has the widest
    # segment
    p = sv.sieve_plan(3 * 10**12, 3 * 10**12 + 2**31)
    assert p["seg_bits"] == 622592 and p["bucket_limit"] == 622592
    assert sv.sieve_plan(3 * 10**12, 3 * 10**12 + 2**31 - 2)["bucket_limit"] == 0
    assert sv.sieve_plan(10**11, 10**11 + 10**6)["bucket_limit"] == 0
    p = sv.sieve_plan(3 * 10**12, 3 * 10**12 + 10**10, tuning=dict(bucket_limit=0xFFFFFFFF))
    assert p["bucket_limit"] == 0 and p["seg_bits"] == 622592
    # any segment size can take buckets (the fill divides by it)
    p = sv.sieve_plan(10**13, 10**13 + 10**9, tuning=dict(seg_bits=491520, bucket_limit=491520))
    assert p["bucket_limit"] == 491520 and p["seg_bits"] == 491520
    # the widest segment can be asked for; anything wider cannot
    assert sv.sieve_plan(2, 10**10, tuning=dict(seg_bits=622592))["seg_bits"] == 622592


@pytest.mark.parametrize("lo,hi,tuning,status", [
    (5, 4, None, -1),
    (0, 10**15 + 1, None, -2),
    (0, 100, dict(seg_bits=1000), -1),
    (0, 100, dict(seg_bits=2**30), -1),
    (0, 100, dict(seg_bits=622592 + 4096), -1),
    (0, 100, dict(seg_bits=1 << 20), -1),
    (0, 100, dict(block_threads=100), -1),
    (0, 100, dict(dense_limit=2**21), -1),
])
def test_plan_errors(lo, hi, tuning, status):
    import paper_1205_4883_amd as sv

    with pytest.raises(sv.SieveError) as e:
        sv.sieve_plan(lo, hi, tuning=tuning)
    assert e.value.status == status


def test_null_context_is_rejected():
    import paper_1205_4883_amd as sv

    lib = sv.sieve._lib()
    pi = ctypes.c_uint64(7)
    assert lib.sieve_range_count(None, 0, 100, ctypes.byref(pi), None) == sv.sieve.SIEVE_EINVAL
    assert pi.value == 7
    assert lib.sieve_range_bitmap(None, 0, 100, None, 0, None, None) == sv.sieve.SIEVE_EINVAL
    assert lib.sieve_batch(None, None, 0, None, 0, None, None) == sv.sieve.SIEVE_EINVAL
    n = ctypes.c_uint64(0)
    assert lib.sieve_base_primes(None, 100, None, 0, ctypes.byref(n)) == sv.sieve.SIEVE_EINVAL
    assert lib.sieve_destroy(None) == 0
    assert lib.sieve_create(None, 0, 0) == sv.sieve.SIEVE_EINVAL
    assert sv.sieve_strerror(-4) == "output buffer too small"


def test_no_device_here_is_enodev():
    import torch

    import paper_1205_4883_amd as sv

    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    with pytest.raises(sv.SieveError) as e:
        sv.sieve_create(0)
    assert e.value.status == sv.sieve.SIEVE_ENODEV


def test_product_code_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_1205_4883_amd")
    for dirpath, _, files in os.walk(pkg):
        for f in files:
            if f.endswith((".py", ".hip", ".h", ".cpp", ".hpp")):
                text = open(os.path.join(dirpath, f)).read()
                assert "oracle" not in text.lower(), os.path.join(dirpath, f)
    hdr = open(os.path.join(ROOT, "include", "sieve.h")).read()
    assert "oracle" not in hdr.lower()
