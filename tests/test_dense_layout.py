"""CPU checks of the committed dense-prime lane layout table against the
script that generates it (spot checks; the full run takes minutes)."""
import os
import re

import numpy as np

from paper_1205_4883_amd import gen_dense_layout as gen

HDR = os.path.join(os.path.dirname(gen.__file__), "csrc", "dense_layout.h")


def _table():
    text = open(HDR).read()
    body = text.split("kDenseStride[kDenseStrideCount] = {")[1].split("};")[0]
    count = int(re.search(r"kDenseStrideCount = (\d+);", text).group(1))
    vals = [int(x) for x in re.findall(r"\d+", body)]
    assert len(vals) == count
    return vals


def test_one_odd_stride_per_prime_from_37_below_2048():
    vals = _table()
    primes = [p for p in gen.primes_below(gen.LIMIT) if p >= gen.FIRST_MARKED]
    assert len(vals) == len(primes) and primes[0] == 37
    assert all(1 <= u <= 255 and u % 2 == 1 for u in vals)


def test_every_odd_stride_gives_each_class_once():
    for u in range(1, 256, 2):
        ks = sorted((u * (l + 64 * j)) % 256 for l in range(64) for j in range(4))
        assert ks == list(range(256))


def test_spot_check_choices_against_the_cost_model():
    vals = _table()
    primes = [p for p in gen.primes_below(gen.LIMIT) if p >= gen.FIRST_MARKED]
    for p in (37, 43, 409, 1021):
        i = primes.index(p)
        cost = gen.layout_cost(p)
        assert vals[i] == int(gen.US[int(np.argmin(cost))]), p
        assert cost[int(np.argmin(cost))] <= cost[0]
