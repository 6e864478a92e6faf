"""GPU tests of the serving loop: every result in the mix equals the same
request sieved alone (plain launch), and equals the oracle on a sample."""
import time

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv():
    import torch

    import paper_1205_4883_amd as sv

    assert torch.cuda.is_available()
    return sv


@pytest.fixture(scope="module")
def alone(sv):
    s = sv.Sieve(0)
    yield s
    s.close()


def _requests(seed, n, max_len=1e7):
    rng = np.random.default_rng(seed)
    lo = np.floor(np.exp(rng.uniform(np.log(1e3), np.log(1e12), n))).astype(np.uint64)
    ln = np.floor(np.exp(rng.uniform(np.log(1e3), np.log(max_len), n))).astype(np.uint64)
    bm = rng.random(n) < 0.5
    return lo, lo + ln, bm


def _drain(server, n, timeout_s=60):
    got = {}
    t0 = time.time()
    while len(got) < n:
        for r in server.results(wait_us=2000):
            got[r["id"]] = r
        assert time.time() - t0 < timeout_s, f"only {len(got)} of {n} results"
    return got


def _check_against_alone(alone, lo, hi, bm, ids, got):
    for i in range(len(lo)):
        r = got[ids[i]]
        assert r["status"] == 0
        words, pi = alone.bitmap(int(lo[i]), int(hi[i]))
        assert r["pi"] == pi, (i, int(lo[i]), int(hi[i]))
        if bm[i]:
            assert np.array_equal(r["words"], words.cpu().numpy().view(np.uint32)), i
        else:
            assert r["words"] is None


def test_server_mix_equals_alone_and_oracle(sv, alone, oracle_mod):
    lo, hi, bm = _requests(21, 300)
    server = sv.Server(0, lanes=3)
    try:
        print("case server mix of 300", flush=True)
        ids = [server.submit(int(a), int(b), bool(f)) for a, b, f in zip(lo, hi, bm)]
        got = _drain(server, len(ids))
        st = server.stats()
        assert st["completed"] == 300
        # requests were batched, lanes overlapped, and no graph was captured
        # while serving (both variants are captured when the server starts)
        assert st["max_batch_seen"] > 1 and st["max_inflight"] >= 2, st
        assert st["graph_captures"] == 0, st
    finally:
        server.close()
    _check_against_alone(alone, lo, hi, bm, ids, got)
    for i in range(0, 300, 10):
        assert got[ids[i]]["pi"] == oracle_mod.count(int(lo[i]), int(hi[i]))


def test_server_single_requests_take_the_plain_launch(sv, alone, oracle_mod):
    # requests submitted one at a time form batches of one, which go through
    # the plain range launch (count published to the lane's pinned word);
    # bucketed and empty ranges fall back to the batch launch
    lo, hi, bm = _requests(31, 40)
    extra = [(10**12 - 10**6, 10**12 + 3 * 10**6, True),
             (10**12, 10**12, False), (7, 7, True), (0, 3, True)]  # empty ranges: batch path
    server = sv.Server(0, lanes=2)
    try:
        ids, got = [], {}
        for i in range(len(lo)):
            ids.append(server.submit(int(lo[i]), int(hi[i]), bool(bm[i])))
            got.update(_drain(server, 1))
        _check_against_alone(alone, lo, hi, bm, ids, got)
        for (a, b, w) in extra:
            rid = server.submit(a, b, w)
            r = _drain(server, 1)[rid]
            assert r["status"] == 0 and r["pi"] == oracle_mod.count(a, b), (a, b)
            if w and b // 2 - a // 2 > 0:
                assert np.array_equal(r["words"], oracle_mod.bitmap(a, b)[0]), (a, b)
        st = server.stats()
        assert st["single_launches"] >= len(lo) + 2
        assert st["batches"] >= st["single_launches"] + 2
    finally:
        server.close()


def test_server_small_batches_as_plain_launches(sv, alone, oracle_mod):
    # A batch of two to eight requests goes as plain launches, one after
    # another on the lane's stream, each count published to its own pinned
    # word and each bitmap copied back by the copy kernel: submitted in
    # groups of five to a one-lane server, the groups become such batches
    # (the first request of a group may leave alone), and every result
    # equals the oracle.
    lo, hi, bm = _requests(51, 40, max_len=3e7)
    server = sv.Server(0, lanes=1)
    try:
        ids, got = [], {}
        print("case server small batches (8 groups of 5)", flush=True)
        for g in range(0, 40, 5):
            ids += [server.submit(int(lo[i]), int(hi[i]), bool(bm[i])) for i in range(g, g + 5)]
            got.update(_drain(server, len(ids) - len(got)))
        st = server.stats()
        assert st["completed"] == 40 and st["graph_captures"] == 0
        assert st["max_batch_seen"] >= 2, st
        assert st["single_launches"] == st["batches"], st  # no batch graph was needed
    finally:
        server.close()
    for i in range(40):
        r = got[ids[i]]
        assert r["status"] == 0
        if bm[i]:
            want, want_pi = oracle_mod.bitmap(int(lo[i]), int(hi[i]))
            assert r["pi"] == want_pi and np.array_equal(r["words"], want), i
        else:
            assert r["pi"] == oracle_mod.count(int(lo[i]), int(hi[i])), i


def test_server_budget_binds_device_memory(sv, alone):
    # The HBM budget is real memory: 64 MiB for the context, each lane's
    # batch buffers, and the rest as the device pool the admitted bitmaps
    # live in.  A budget about 10 MiB over the fixed part leaves a pool far
    # smaller than the 60 bitmaps below (125 KB .. 1 MB each, 34 MB in
    # all): admission must wait for earlier requests to finish, the pool is
    # never over-committed, and every result stays exact.
    import torch

    budget = (64 + 2 + 10) << 20
    rng = np.random.default_rng(5)
    lo = rng.integers(10**9, 10**11, 60).astype(np.uint64)
    hi = lo + rng.integers(2 * 10**6, 16 * 10**6, 60).astype(np.uint64)
    bm = np.ones(60, dtype=bool)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info(0)[0]
    server = sv.Server(0, lanes=2, hbm_budget_bytes=budget, host_arena_bytes=1 << 22)
    try:
        held = free0 - torch.cuda.mem_get_info(0)[0]
        print(f"case server budget: {budget} budget, {held} device bytes taken by the server", flush=True)
        assert held <= budget + (32 << 20)  # the runtime's own stream and queue memory aside
        ids = [server.submit(int(a), int(b), True) for a, b in zip(lo, hi)]
        got = _drain(server, len(ids))
        st = server.stats()
        assert 0 < st["device_pool_bytes"] <= budget - (64 << 20)
        assert st["deferred"] > 0
        assert 0 < st["peak_admitted_bytes"] <= st["device_pool_bytes"]
        assert st["peak_host_bytes"] <= 1 << 22
        assert st["graph_captures"] == 0
    finally:
        server.close()
    _check_against_alone(alone, lo, hi, bm, ids, got)


def test_server_budget_below_the_fixed_memory_is_refused(sv):
    with pytest.raises(sv.SieveError) as e:
        sv.Server(0, hbm_budget_bytes=1 << 20)
    assert e.value.status == sv.sieve.SIEVE_ENOMEM


def test_server_staggered_arrivals_equal_alone_and_oracle(sv, alone, oracle_mod):
    # Requests arrive in waves while earlier ones are on the GPU, including
    # ranges of the served workload's greatest length (about 1e9 integers,
    # bitmaps of 62.5 MB); every result equals the same range sieved alone,
    # word for word, and a sample equals the oracle.
    rng = np.random.default_rng(41)
    lo, hi, bm = _requests(43, 96, max_len=1e8)
    lo = np.concatenate([lo, np.array([10**12 - 10**9 - 12345, 3 * 10**11 + 1, 10**9], dtype=np.uint64)])
    hi = np.concatenate([hi, np.array([10**12 - 12345, 3 * 10**11 + 1 + 999_999_937, 2 * 10**9],
                                      dtype=np.uint64)])
    bm = np.concatenate([bm, np.array([True, True, False])])
    order = rng.permutation(lo.size)
    server = sv.Server(0, lanes=3)
    try:
        ids, got = {}, {}
        print(f"case server staggered arrivals ({lo.size} requests)", flush=True)
        for wave in np.array_split(order, 12):
            for i in wave:
                ids[int(i)] = server.submit(int(lo[i]), int(hi[i]), bool(bm[i]))
            for r in server.results(wait_us=300):
                got[r["id"]] = r
        got.update(_drain(server, lo.size - len(got), timeout_s=120))
        st = server.stats()
        assert st["completed"] == lo.size and st["graph_captures"] == 0
        assert st["max_inflight"] >= 2, st
    finally:
        server.close()
    rs = [got[ids[i]] for i in range(lo.size)]
    # some request was admitted while another was on the device
    assert any(a["t_admit_ns"] > b["t_launch_ns"] and a["t_admit_ns"] < b["t_done_ns"]
               for a in rs for b in rs if a["id"] != b["id"])
    _check_against_alone(alone, lo, hi, bm, [ids[i] for i in range(lo.size)], got)
    for i in list(range(0, lo.size, 8)) + [lo.size - 3, lo.size - 2, lo.size - 1]:
        r = got[ids[i]]
        if bm[i]:
            want, want_pi = oracle_mod.bitmap(int(lo[i]), int(hi[i]))
            assert r["pi"] == want_pi and np.array_equal(r["words"], want), i
        else:
            assert r["pi"] == oracle_mod.count(int(lo[i]), int(hi[i])), i


def test_server_plain_mode_matches(sv, alone):
    lo, hi, bm = _requests(33, 60)
    server = sv.Server(0, mode=sv.sieve.SIEVE_SERVE_PLAIN)
    try:
        ids = [server.submit(int(a), int(b), bool(f)) for a, b, f in zip(lo, hi, bm)]
        got = _drain(server, len(ids))
        assert server.stats()["max_batch_seen"] == 1
    finally:
        server.close()
    _check_against_alone(alone, lo, hi, bm, ids, got)


def test_server_argument_errors(sv):
    server = sv.Server(0, max_batch_words=1024)
    try:
        with pytest.raises(sv.SieveError) as e:
            server.submit(10, 5)
        assert e.value.status == sv.sieve.SIEVE_EINVAL
        with pytest.raises(sv.SieveError) as e:
            server.submit(0, 10**15 + 1)
        assert e.value.status == sv.sieve.SIEVE_ERANGE
        with pytest.raises(sv.SieveError) as e:
            server.submit(0, 10**6, bitmap=True)  # 15625 words > 1024 per batch
        assert e.value.status == sv.sieve.SIEVE_ENOMEM
        rid = server.submit(0, 10**6, bitmap=False)  # count only: no words needed
        got = _drain(server, 1)
        assert got[rid]["pi"] == 78498
        with pytest.raises(sv.SieveError):
            sv.sieve_server_release(server.srv, 987654321)
    finally:
        server.close()


def test_serve_trace_batched_equals_plain_and_oracle(sv, oracle_mod):
    from paper_1205_4883_amd import workloads

    tr = workloads.serve_trace(1, seconds=1.0)
    n = tr["t"].size
    flags = tr["bitmap"].astype(np.uint32)
    print(f"case serve trace 1 s ({n} requests)", flush=True)
    pi_b, lat_b, st_b = sv.sieve_serve_trace(0, tr["lo"], tr["hi"], flags, tr["t"])
    pi_p, lat_p, st_p = sv.sieve_serve_trace(0, tr["lo"], tr["hi"], flags, tr["t"],
                                             mode=sv.sieve.SIEVE_SERVE_PLAIN)
    assert st_b["completed"] == n and st_p["completed"] == n
    assert st_b["graph_captures"] == 0
    assert np.array_equal(pi_b, pi_p)
    assert np.all(lat_b > 0) and np.all(lat_p > 0)
    for i in range(0, n, 100):
        assert int(pi_b[i]) == oracle_mod.count(int(tr["lo"][i]), int(tr["hi"][i])), i
