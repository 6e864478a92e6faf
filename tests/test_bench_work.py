"""CPU checks of the algorithmic work figures the benchmark prices its roofline
with: closed-form counts of crossed-off odd multiples against enumeration."""
import math

import numpy as np
import pytest

import bench


def _primes_upto(n):
    s = np.ones(n + 1, dtype=bool)
    s[:2] = False
    for i in range(2, math.isqrt(n) + 1):
        if s[i]:
            s[i * i::i] = False
    return np.nonzero(s)[0].astype(np.uint32)


def _enumerated_marks(lo, hi, pmin):
    """Every odd m in [lo, hi) crossed off by a prime pmin <= p with p^2 <= m,
    counted once per such prime (the sieve's atomic updates)."""
    n = 0
    for p in _primes_upto(max(math.isqrt(max(hi - 1, 0)), 2)).tolist():
        if p < pmin or p * p > hi - 1:
            continue
        for m in range(max(p * p, lo), hi):
            if m % p == 0 and m % 2 == 1:
                n += 1
    return n


@pytest.mark.parametrize("lo,hi", [(0, 1), (2, 3), (0, 2000), (2, 10007), (1369, 1370),
                                   (999, 5000), (40000, 47321), (123457, 130000)])
def test_marks_match_enumeration(lo, hi):
    primes = _primes_upto(1000)
    for pmin in (7, 37):
        marks, lane_ops, words = bench.algorithmic_lds_ops(primes, lo, hi, pmin=pmin)
        assert marks == _enumerated_marks(lo, hi, pmin)
        assert words == (hi // 2 - lo // 2 + 31) // 32
        assert lane_ops == marks + 2 * words
    roof = bench.lds_roofline(primes, [(lo, hi)], 1.0)
    w = roof["work_per_launch"]
    assert w["marks"] == _enumerated_marks(lo, hi, 37)
    assert w["marks_wheel30"] == _enumerated_marks(lo, hi, 7)


def _enumerated_issued(lo, hi):
    """The atomics the kernels issue: odd m in [lo, hi), m = p*k with
    p >= 37, p^2 <= m and k prime to 30, once per such prime."""
    n = 0
    for p in _primes_upto(max(math.isqrt(max(hi - 1, 0)), 2)).tolist():
        if p < 37 or p * p > hi - 1:
            continue
        for m in range(max(p * p, lo), hi):
            if m % p == 0 and math.gcd(m // p, 30) == 1:
                n += 1
    return n


@pytest.mark.parametrize("lo,hi", [(0, 2000), (2, 10007), (1369, 1370), (40000, 47321), (123457, 130000)])
def test_issued_marks_match_enumeration(lo, hi):
    primes = _primes_upto(1000)
    roof = bench.lds_roofline(primes, [(lo, hi)], 1.0)
    w = roof["work_per_launch"]
    assert w["issued_marks"] == _enumerated_issued(lo, hi)
    assert w["issued_lds_lane_ops"] == w["issued_marks"] + bench.ISSUED_OPS_PER_WORD * w["words"]
    assert w["issued_marks"] <= w["marks"]


def test_roofline_sums_over_intervals():
    primes = _primes_upto(2000)
    ivs = [(10**6, 10**6 + 3001), (5, 5), (2, 99991), (3 * 10**6, 3 * 10**6 + 64)]
    roof = bench.lds_roofline(primes, ivs, 2.0)
    w = roof["work_per_launch"]
    assert w["marks"] == sum(bench.algorithmic_lds_ops(primes, a, b)[0] for a, b in ivs)
    assert w["marks_wheel30"] == sum(bench.algorithmic_lds_ops(primes, a, b, pmin=7)[0]
                                     for a, b in ivs)
    assert w["lds_lane_ops"] == w["marks"] + 2 * w["words"]
    assert roof["frac"] == pytest.approx(w["lds_lane_ops"] / 2.0 / bench.LDS_PEAK_LANE_OPS)
    assert w["lds_lane_ops_wheel30"] >= w["lds_lane_ops"] >= w["issued_lds_lane_ops"] - 3 * w["words"]
    assert "frac_wheel30" not in roof  # the wheel-30 work is reported, not priced


def test_presieve_set_is_the_odd_primes_below_the_first_marked_one():
    assert bench.PRESIEVE_PRIMES == [p for p in _primes_upto(bench.FIRST_MARKED_PRIME - 1).tolist()
                                     if p > 2]


def test_committed_counter_runs_are_sane():
    # the rocprofv3 byte counts behind the roofline's traffic figures must
    # at least cover the output each launch writes, and a count-only launch
    # must write far less than the bitmap it never stores
    import json
    import os

    prof = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "profiles")

    def rec(name):
        with open(os.path.join(prof, f"traffic_{name}.json")) as f:
            return json.load(f)

    bitmap = rec("bitmap-1e9")
    assert bitmap["hbm_write_bytes_per_launch"] >= 4 * 15_625_000
    assert bitmap["hbm_write_bytes_per_launch"] < 2 * 4 * 15_625_000
    batch = rec("batch-4096")
    assert batch["hbm_write_bytes_per_launch"] >= 2_801_070_496
    count = rec("count-1e10")
    assert count["hbm_write_bytes_per_launch"] < 0.05 * 4 * 156_250_000
    for r in (bitmap, batch, count):
        cal = r["copy_calibration"]
        # the copy kernel reads and writes 256 MiB: both scales near 1 or 2
        assert 0.9 < cal["write_scale"] < 2.1 and 0.9 < cal["fetch_scale"] < 2.1
