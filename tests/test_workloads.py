"""CPU checks of the seeded workload generators (inputs only, no sieve)."""
import numpy as np

from paper_1205_4883_amd import workloads


def test_batch_intervals_seed0_facts():
    lo, hi = workloads.batch_intervals(0)
    L = hi - lo
    assert lo.size == 4096 and lo.dtype == np.uint64
    assert int(L.sum()) == 44817000774
    assert int(L.min()) == 10009 and int(L.max()) == 99997022
    assert int(lo.min()) >= 10**6 and int(hi.max()) < 10**12
    nw = (hi // 2 - lo // 2 + 31) // 32
    assert int(4 * nw.sum()) == 2801070496
    assert workloads.fingerprint(lo, hi).startswith("151a0f3204e6595a")


def test_serve_trace_seed1_shape():
    tr = workloads.serve_trace(1)
    n = tr["t"].size
    assert 119000 < n < 121000  # 2000 req/s for 60 s
    assert np.all(np.diff(tr["t"]) >= 0) and tr["t"][-1] < 60.0
    ln = tr["hi"] - tr["lo"]
    assert int(ln.min()) >= 1000 and int(ln.max()) < 10**9
    assert int(tr["lo"].min()) >= 1000 and int(tr["hi"].max()) <= 10**12 + 10**9
    assert 0.49 < tr["bitmap"].mean() < 0.51
    assert workloads.fingerprint(tr["lo"], tr["hi"]).startswith("ece10d7e10645d50")


def test_generators_are_deterministic():
    a = workloads.batch_intervals(0)
    b = workloads.batch_intervals(0)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[1], b[1])
    assert not np.array_equal(workloads.batch_intervals(1)[0], a[0])
