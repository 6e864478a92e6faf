"""CPU check of the bucket fill's segment split for segments that are not a
power of two: the float quotient o * (1 / seg_bits), truncated, is within one
of o // seg_bits for every bit offset o of a chunk of 32 segments, and one
correction step makes it exact.  numpy's float32 multiply and conversion round
as the device's v_mul_f32 (round to nearest) and v_cvt_u32_f32 (truncation)
do."""
import numpy as np
import pytest

CHUNK = 32  # segments per fill workgroup


def split(o, seg_bits):
    rcp = np.float32(1.0) / np.float32(seg_bits)
    q = (o.astype(np.float32) * rcp).astype(np.int64)
    b = q * seg_bits
    hi = b > o
    q = np.where(hi, q - 1, q)
    b = np.where(hi, b - seg_bits, b)
    lo = (o - b) >= seg_bits
    q = np.where(lo, q + 1, q)
    b = np.where(lo, b + seg_bits, b)
    return q, o - b


@pytest.mark.parametrize("seg_bits", [622592, 491520, 15360 * 32, 327680, 96, 32 * 33, 1 << 20])
def test_float_split_is_exact_over_a_chunk(seg_bits):
    o = np.arange(CHUNK * seg_bits, dtype=np.int64)
    q, off = split(o, seg_bits)
    assert np.array_equal(q, o // seg_bits)
    assert np.array_equal(off, o % seg_bits)


def test_raw_quotient_is_off_by_at_most_one():
    # the correction handles both directions, and is needed for the widest
    # segment (the bare truncated quotient is off by one at some offsets)
    seg_bits = 622592
    o = np.arange(CHUNK * seg_bits, dtype=np.int64)
    q = (o.astype(np.float32) * (np.float32(1.0) / np.float32(seg_bits))).astype(np.int64)
    err = q - o // seg_bits
    assert err.min() >= -1 and err.max() <= 1 and np.any(err != 0)
