"""GPU parity: the HIP path through the C ABI against the CPU oracle.

Every comparison is exact (bitmaps word for word, counts as integers): the
sieve's result is a set of integers with one correct value per range
(paper, Sections 1 and 3.1), so there is no tolerance.
"""
import random

import numpy as np
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sv_mod():
    import paper_1205_4883_amd as sv

    return sv


@pytest.fixture(scope="module")
def gpu(sv_mod):
    import torch

    assert torch.cuda.is_available()
    s = sv_mod.Sieve(0)
    yield s
    s.close()


def _cmp_bitmap(gpu, oracle_mod, lo, hi, threads=None):
    print(f"case bitmap [{lo}, {hi})", flush=True)
    words, pi = gpu.bitmap(lo, hi)
    got = words.cpu().numpy().view(np.uint32)
    ref, ref_pi = oracle_mod.bitmap(lo, hi, threads=threads)
    assert pi == ref_pi, (lo, hi, pi, ref_pi)
    if not np.array_equal(got, ref):
        bad = np.nonzero(got != ref)[0]
        raise AssertionError(f"[{lo},{hi}): {bad.size} words differ, first {bad[:5]} "
                             f"got {got[bad[:5]]} want {ref[bad[:5]]}")
    assert gpu.count(lo, hi) == ref_pi
    return pi


# -- the three single-range workloads at full size ----------------------------

def test_c1_bitmap_2_to_1e7(gpu, oracle_mod):
    assert _cmp_bitmap(gpu, oracle_mod, 2, 10**7) == 664579


def test_c2_bitmap_2_to_1e9(gpu, oracle_mod):
    assert _cmp_bitmap(gpu, oracle_mod, 2, 10**9) == 50847534


def test_c3_count_2_to_1e10(gpu, oracle_mod):
    print("case count [2, 1e10)", flush=True)
    pi = gpu.count(2, 10**10)
    assert pi == 455052511
    assert pi == oracle_mod.count(2, 10**10)


def test_c3_sampled_bits_at_full_size(gpu, oracle_mod):
    # the count-only launch of [2, 1e10) writes no bitmap; sample the
    # bitmap launch of the same range at scattered windows
    print("case sampled bitmap [2, 1e10)", flush=True)
    lo, hi = 2, 10**10
    n = gpu.torch.cuda
    words, pi = gpu.bitmap(lo, hi)
    assert pi == 455052511
    rng = random.Random(11)
    for _ in range(24):
        w0 = rng.randrange(0, words.numel() - 2048)
        a = 2 + 64 * w0  # [a, a + 64*2048) has bit 0 at a + 1 = 3 + 64*w0
        got = words[w0:w0 + 2048].cpu().numpy().view(np.uint32)
        ref, _ = oracle_mod.bitmap(a, a + 64 * 2048)
        assert np.array_equal(got, ref[:2048]), w0
    del words
    n.empty_cache()


# -- small and edge ranges ----------------------------------------------------

def test_every_tiny_range(gpu, oracle_mod):
    print("case all ranges in [0, 130]", flush=True)
    for lo in range(0, 131):
        for hi in range(lo, 131):
            words, pi = gpu.bitmap(lo, hi)
            ref, ref_pi = oracle_mod.bitmap(lo, hi)
            assert pi == ref_pi, (lo, hi)
            assert np.array_equal(words.cpu().numpy().view(np.uint32), ref), (lo, hi)


@pytest.mark.parametrize("lo,hi", [
    (0, 1), (0, 2), (0, 3), (1, 3), (2, 3), (3, 4), (0, 8), (2, 8), (5, 6), (4, 5),
    (0, 121), (0, 122), (120, 122), (0, 961), (0, 962), (0, 1369), (0, 1370),
    (999999999989, 999999999990), (999999999990, 1000000000039),
    (999999999990, 1000000000040), (10**12 - 10**6, 10**12 + 10**6),
    (10**15 - 3 * 10**6, 10**15), (10**15 - 1, 10**15),
])
def test_edge_ranges(gpu, oracle_mod, lo, hi):
    _cmp_bitmap(gpu, oracle_mod, lo, hi)


def test_known_endpoint_counts(gpu):
    assert gpu.count(999999999990, 1000000000039) == 0
    assert gpu.count(999999999990, 1000000000040) == 1
    assert gpu.count(999999999989, 999999999990) == 1
    assert gpu.count(0, 2**32) == 203280221
    for n in [561, 1105, 1729, 2465, 2821, 6601, 8911]:
        assert gpu.count(n, n + 1) == 0


@pytest.mark.parametrize("seed", range(6))
def test_random_ranges_across_magnitudes(gpu, oracle_mod, seed):
    rng = random.Random(100 + seed)
    for _ in range(6):
        e = rng.uniform(2, 15)
        lo = min(int(10**e), 10**15 - 1)
        ln = int(10 ** rng.uniform(0, 6.7))
        hi = min(lo + ln, 10**15)
        _cmp_bitmap(gpu, oracle_mod, lo, hi)


def test_segment_boundary_straddles(gpu, oracle_mod):
    # plan the segment size, then cut ranges at +-1 around segment edges
    import paper_1205_4883_amd as sv

    gpu.tuning(seg_bits=4096, dense_limit=0, block_threads=256)
    try:
        base = 10**11
        seg_ints = 2 * 4096
        for k in [1, 2, 7]:
            for d in [-3, -2, -1, 0, 1, 2, 3]:
                lo = base
                hi = base + k * seg_ints + d
                _cmp_bitmap(gpu, oracle_mod, lo, hi)
                _cmp_bitmap(gpu, oracle_mod, lo + 1, hi)
    finally:
        gpu.tuning(seg_bits=0, dense_limit=0, block_threads=0)
    assert sv.sieve_get_tuning(gpu.ctx)["seg_bits"] == 0


@pytest.mark.parametrize("seg_bits,dense_limit,threads", [
    (4096, 37, 256), (4096, 64, 512), (32768, 0, 1024), (131072, 37, 256),
    (524288, 0, 1024), (524288, 37, 1024), (524288, 2**20, 1024), (262144, 1000, 512),
    (622592, 0, 1024), (622592, 2048, 1024),
])
def test_tuning_sweep(gpu, oracle_mod, seg_bits, dense_limit, threads):
    gpu.tuning(seg_bits=seg_bits, dense_limit=dense_limit, block_threads=threads)
    try:
        for lo, hi in [(0, 3 * 10**6 + 17), (10**10 - 777, 10**10 + 5 * 10**6),
                       (10**13 + 1, 10**13 + 2 * 10**6 + 3)]:
            _cmp_bitmap(gpu, oracle_mod, lo, hi)
        assert gpu.count(2, 10**9) == 50847534
    finally:
        gpu.tuning(seg_bits=0, dense_limit=0, block_threads=0)


@pytest.mark.parametrize("lo,hi,seg_bits,threads,dense_limit", [
    (2, 2 * 10**8, 4096, 256, 0),             # carried primes whose p*p falls inside a run
    (10**9 + 3, 10**9 + 2 * 10**8, 4096, 512, 0),
    (0, 3 * 10**8, 16384, 1024, 37),          # no dense primes: every prime carried or scanned
    (10**12 + 1, 10**12 + 4 * 10**8, 8192, 256, 0),  # runs inside bucket windows
    # 16 waves: inside runs only waves 0..7 take dense primes, and the
    # uncarried sparse primes are shared out from the LDS counter
    (10**9 + 3, 10**9 + 3 * 10**8 + 7, 16384, 1024, 0),
    (3 * 10**10, 3 * 10**10 + 3 * 10**8, 16384, 1024, 600),
])
def test_runs_of_segments_with_carried_offsets(gpu, oracle_mod, sv_mod, lo, hi, seg_bits, threads,
                                               dense_limit):
    # small segments give launches with many more segments than workgroups, so
    # work items are runs of consecutive segments and lanes carry their
    # primes' next multiples from segment to segment
    gpu.tuning(seg_bits=seg_bits, block_threads=threads, dense_limit=dense_limit)
    try:
        plan = sv_mod.sieve_plan(lo, hi, tuning=gpu.tuning())
        assert plan["n_segments"] > 9000
        _cmp_bitmap(gpu, oracle_mod, lo, hi)
    finally:
        gpu.tuning(seg_bits=0, block_threads=0, dense_limit=0)


def test_additivity_on_gpu(gpu):
    rng = random.Random(7)
    for _ in range(30):
        a = rng.randrange(0, 10**12)
        c = a + rng.randrange(0, 5 * 10**7)
        b = rng.randrange(a, c + 1)
        assert gpu.count(a, c) == gpu.count(a, b) + gpu.count(b, c)


def test_properties_of_a_large_range_near_the_top(gpu, oracle_mod):
    # at a size the oracle is not run on whole: [1e15 - 2^33, 1e15) (2^32
    # odd integers, 512 MiB of bitmap).  The words of [a, b) and [b, c) (b at
    # a multiple of 64 from a) concatenate to those of [a, c); the count
    # equals the bitmap's popcount; twelve sampled 2048-word windows equal
    # the oracle's bitmap of the same integers; and sampled set bits are
    # prime and sampled clear bits composite by Miller-Rabin.
    print("case large-range properties below 1e15", flush=True)
    torch = gpu.torch
    a, c = 10**15 - 2**33, 10**15
    b = a + 64 * 50_000_017
    w_ac, pi_ac = gpu.bitmap(a, c)
    w_ab, pi_ab = gpu.bitmap(a, b)
    w_bc, pi_bc = gpu.bitmap(b, c)
    assert pi_ac == pi_ab + pi_bc == gpu.count(a, c)
    assert torch.equal(w_ac, torch.cat([w_ab, w_bc]))
    del w_ab, w_bc
    # popcount in chunks (the whole bitmap as int64 bit counts would need GBs)
    total = 0
    u8 = w_ac.view(torch.uint8)
    table = torch.tensor([bin(i).count("1") for i in range(256)], dtype=torch.int64, device=w_ac.device)
    for k in range(0, u8.numel(), 1 << 26):
        total += int(table[u8[k:k + (1 << 26)].long()].sum())
    assert total == pi_ac  # no 2 in range
    rng = random.Random(17)
    words = w_ac.cpu().numpy().view(np.uint32)
    starts = [0, words.size - 2048] + [rng.randrange(0, words.size - 2048) for _ in range(10)]
    for w0 in starts:
        lo_w = a + 64 * w0
        hi_w = min(c, lo_w + 64 * 2048)
        ref, _ = oracle_mod.bitmap(lo_w, hi_w)
        assert np.array_equal(words[w0:w0 + ref.size], ref), (lo_w, hi_w)
    ns, want = [], []
    base = (a & ~1) + 1
    for _ in range(4000):
        i = rng.randrange(0, words.size * 32)
        n = base + 2 * i
        if n >= c:
            continue
        ns.append(n)
        want.append(bool((words[i >> 5] >> (i & 31)) & 1))
    assert any(want) and not all(want)
    got = gpu.is_prime(ns)
    assert got.tolist() == want
    del w_ac
    torch.cuda.empty_cache()


# -- base primes -------------------------------------------------------------

@pytest.mark.parametrize("limit", [0, 1, 2, 3, 100, 65535, 65536, 100000, 2**20, 3 * 10**6, 31622777])
def test_base_primes(gpu, oracle_mod, limit):
    got = gpu.base_primes(limit)
    ref = oracle_mod.base_primes(limit)
    assert np.array_equal(got, ref)


# -- ABI behaviour on the device ---------------------------------------------

def test_errors_leave_outputs_untouched(gpu, sv_mod):
    import torch

    buf = torch.full((8,), -1, dtype=torch.int32, device="cuda:0")
    with pytest.raises(sv_mod.SieveError) as e:
        sv_mod.sieve_range_bitmap(gpu.ctx, 0, 1000, buf, 8)  # needs 16 words
    assert e.value.status == sv_mod.sieve.SIEVE_EBUFSZ
    with pytest.raises(sv_mod.SieveError) as e:
        sv_mod.sieve_range_bitmap(gpu.ctx, 100, 10, buf, 8)
    assert e.value.status == sv_mod.sieve.SIEVE_EINVAL
    with pytest.raises(sv_mod.SieveError) as e:
        sv_mod.sieve_range_count(gpu.ctx, 0, 10**15 + 1)
    assert e.value.status == sv_mod.sieve.SIEVE_ERANGE
    with pytest.raises(sv_mod.SieveError) as e:
        sv_mod.sieve_range_bitmap(gpu.ctx, 0, 100, buf.data_ptr() + 2, 4)
    assert e.value.status == sv_mod.sieve.SIEVE_EINVAL
    torch.cuda.synchronize()
    assert (buf.cpu() == -1).all()
    assert sv_mod.sieve_range_count(gpu.ctx, 10, 10) == 0
    assert sv_mod.sieve_range_count(gpu.ctx, 2, 2) == 0


def test_bitmap_leaves_words_past_the_range(gpu, oracle_mod, sv_mod):
    import torch

    buf = torch.full((200,), 0x5A5A5A5A, dtype=torch.int32, device="cuda:0")
    pi = sv_mod.sieve_range_bitmap(gpu.ctx, 1000, 1000 + 64 * 100 - 30, buf, 200)
    ref, ref_pi = oracle_mod.bitmap(1000, 1000 + 64 * 100 - 30)
    host = buf.cpu().numpy().view(np.uint32)
    assert pi == ref_pi
    assert np.array_equal(host[:100], ref)
    assert (host[100:] == 0x5A5A5A5A).all()


def test_async_bitmap_on_torch_stream(gpu, oracle_mod, sv_mod):
    import torch

    lo, hi = 10**11, 10**11 + 10**7
    out = gpu.alloc_words(lo, hi)
    st = torch.cuda.Stream()
    with torch.cuda.stream(st):
        sv_mod.sieve_range_bitmap(gpu.ctx, lo, hi, out, out.numel(), want_pi=False, stream=st)
        host = out.cpu()  # ordered after the sieve on the same stream
    st.synchronize()
    ref, _ = oracle_mod.bitmap(lo, hi)
    assert np.array_equal(host.numpy().view(np.uint32), ref)


# -- batch -----------------------------------------------------------------

def test_batch_matches_oracle(gpu, oracle_mod):
    rng = np.random.default_rng(3)
    n = 300
    los = np.floor(np.exp(rng.uniform(np.log(1), np.log(1e12), n))).astype(np.uint64)
    lens = np.floor(np.exp(rng.uniform(np.log(1), np.log(3e6), n))).astype(np.uint64)
    his = los + lens
    los[:5] = [0, 1, 2, 3, 5]
    his[:5] = [0, 2, 3, 1000, 1_000_003]
    print(f"case batch of {n}", flush=True)
    pi, words, offs = gpu.batch(los, his, want_bitmap=True)
    host = words.cpu().numpy().view(np.uint32)
    for i in range(n):
        lo, hi = int(los[i]), int(his[i])
        ref, ref_pi = oracle_mod.bitmap(lo, hi)
        assert int(pi[i]) == ref_pi, (i, lo, hi)
        o = int(offs[i])
        assert np.array_equal(host[o:o + ref.size], ref), (i, lo, hi)
    pi2 = gpu.batch(los, his, want_bitmap=False)
    assert np.array_equal(pi, pi2)


def test_batch_near_the_top_of_the_domain(gpu, oracle_mod):
    # intervals up to SIEVE_MAX_HI need base primes up to 31,622,776 (the
    # batch kernel scans them all per segment, no buckets)
    los = np.array([10**15 - 3 * 10**6, 10**15 - 10**5 - 1, 9 * 10**14 + 7, 10**15 - 64], dtype=np.uint64)
    his = np.array([10**15, 10**15 - 10**5 + 12345, 9 * 10**14 + 2 * 10**6, 10**15], dtype=np.uint64)
    print("case batch near 1e15", flush=True)
    pi, words, offs = gpu.batch(los, his, want_bitmap=True)
    host = words.cpu().numpy().view(np.uint32)
    for i in range(len(los)):
        ref, ref_pi = oracle_mod.bitmap(int(los[i]), int(his[i]))
        assert int(pi[i]) == ref_pi, i
        o = int(offs[i])
        assert np.array_equal(host[o:o + ref.size], ref), i


def test_async_bitmaps_on_several_streams(gpu, oracle_mod, sv_mod):
    # asynchronous calls on different streams overlap on the device; each must
    # keep its own segment queue
    import torch

    ranges = [(10**9 + 17 * k * 10**6, 10**9 + 17 * k * 10**6 + 3 * 10**6 + k) for k in range(20)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    outs = []
    for k, (lo, hi) in enumerate(ranges):
        st = streams[k % 4]
        out = gpu.alloc_words(lo, hi)
        with torch.cuda.stream(st):
            sv_mod.sieve_range_bitmap(gpu.ctx, lo, hi, out, out.numel(), want_pi=False, stream=st)
        outs.append((out, st))
    torch.cuda.synchronize()
    for (lo, hi), (out, _) in zip(ranges, outs):
        ref, _ = oracle_mod.bitmap(lo, hi)
        assert np.array_equal(out.cpu().numpy().view(np.uint32)[:ref.size], ref), (lo, hi)


def test_batch_graph_replays_and_shrinks(gpu, oracle_mod):
    # the captured batch graph is replayed for batches of different sizes
    # (it reads sizes from device memory) and must match the oracle each time
    rng = np.random.default_rng(9)
    for n in [64, 17, 64, 1]:
        los = np.floor(np.exp(rng.uniform(np.log(10), np.log(1e12), n))).astype(np.uint64)
        his = los + np.floor(np.exp(rng.uniform(0, np.log(2e6), n))).astype(np.uint64)
        pi = gpu.batch(los, his, want_bitmap=False)
        for i in range(n):
            assert int(pi[i]) == oracle_mod.count(int(los[i]), int(his[i])), (n, i)


@pytest.mark.parametrize("seg_bits,threads", [(4096, 256), (65536, 256), (622592, 1024)])
def test_batch_tunings(gpu, oracle_mod, seg_bits, threads):
    rng = np.random.default_rng(seg_bits)
    los = np.floor(np.exp(rng.uniform(0, np.log(1e11), 40))).astype(np.uint64)
    his = los + np.floor(np.exp(rng.uniform(0, np.log(3e6), 40))).astype(np.uint64)
    gpu.tuning(seg_bits=seg_bits, block_threads=threads)
    try:
        pi, words, offs = gpu.batch(los, his, want_bitmap=True)
        host = words.cpu().numpy().view(np.uint32)
        for i in range(len(los)):
            ref, ref_pi = oracle_mod.bitmap(int(los[i]), int(his[i]))
            assert int(pi[i]) == ref_pi
            o = int(offs[i])
            assert np.array_equal(host[o:o + ref.size], ref), i
    finally:
        gpu.tuning()
        gpu.tuning(seg_bits=0, block_threads=0)


def test_batch_workload_counts(gpu, oracle_mod):
    # the full 4096-interval batched workload: every count against the oracle
    from paper_1205_4883_amd import workloads

    los, his = workloads.batch_intervals(0)
    print("case batch workload seed 0", flush=True)
    pi = gpu.batch(los, his, want_bitmap=False)
    for i in range(len(los)):
        assert int(pi[i]) == oracle_mod.count(int(los[i]), int(his[i])), i


def test_batch_workload_bitmaps(gpu, oracle_mod):
    # the full 4096-interval batched workload with packed bitmaps (2.8 GB on
    # the device): every interval shorter than 1e6 and a seeded 10% of the
    # rest are compared word for word, and every count against its bitmap
    from paper_1205_4883_amd import workloads

    los, his = workloads.batch_intervals(0)
    print("case batch workload seed 0 with bitmaps", flush=True)
    pi, words, offs = gpu.batch(los, his, want_bitmap=True)
    lens = his - los
    pick = np.zeros(len(los), dtype=bool)
    pick[lens < 10**6] = True
    rest = np.nonzero(~pick)[0]
    pick[np.random.default_rng(12345).choice(rest, size=len(los) // 10, replace=False)] = True
    checked = 0
    for i in np.nonzero(pick)[0]:
        lo, hi = int(los[i]), int(his[i])
        ref, ref_pi = oracle_mod.bitmap(lo, hi)
        o = int(offs[i])
        got = words[o:o + ref.size].cpu().numpy().view(np.uint32)
        assert int(pi[i]) == ref_pi, (i, lo, hi)
        assert np.array_equal(got, ref), (i, lo, hi)
        checked += 1
    assert checked >= 410
    del words


def test_autotune_single_range_and_batch(gpu, oracle_mod, sv_mod):
    # the tuner times its candidates, applies the winner, caches it, and the
    # results under the chosen tuning stay exact
    lo, hi = 10**9, 10**9 + 2 * 10**8
    try:
        t, ms = sv_mod.sieve_autotune(gpu.ctx, [lo], [hi])
        # the automatic plan (zero fields) is one of the candidates; the
        # refinement may then cap the workgroups per CU
        assert ms > 0 and t["seg_bits"] in (0, 1 << 17, 1 << 18, 1 << 19, 622592)
        if t["seg_bits"]:
            assert t["block_threads"] in (512, 1024) and t["dense_limit"] >= 37
        else:
            assert t["block_threads"] == 0 and t["dense_limit"] == 0
        assert t["wg_per_cu"] in (0, 1, 2)
        assert gpu.tuning()["seg_bits"] == t["seg_bits"]
        t2, ms2 = sv_mod.sieve_autotune(gpu.ctx, [lo], [hi], apply=False)
        assert t2 == t and ms2 == ms  # cache hit
        assert gpu.count(lo, hi) == oracle_mod.count(lo, hi)
        rng = np.random.default_rng(21)
        los = np.floor(np.exp(rng.uniform(np.log(1e6), np.log(1e11), 64))).astype(np.uint64)
        his = los + np.floor(np.exp(rng.uniform(np.log(1e4), np.log(1e7), 64))).astype(np.uint64)
        tb, _ = sv_mod.sieve_autotune(gpu.ctx, los, his)
        pi = gpu.batch(los, his)
        for i in range(len(los)):
            assert int(pi[i]) == oracle_mod.count(int(los[i]), int(his[i])), (tb, i)
    finally:
        gpu.tuning(seg_bits=0, dense_limit=0, block_threads=0, wg_per_cu=0, bucket_limit=0)


def test_autotune_bucketed_range(gpu, oracle_mod, sv_mod):
    # high in the domain the automatic plan uses hit buckets, so the tuner
    # also times larger large-prime thresholds and no buckets at all
    lo, hi = 10**13, 10**13 + 2**31
    try:
        gpu.tuning(seg_bits=0, dense_limit=0, block_threads=0, wg_per_cu=0, bucket_limit=0)
        assert sv_mod.sieve_plan(lo, hi, tuning=gpu.tuning())["bucket_limit"] > 0
        t, ms = sv_mod.sieve_autotune(gpu.ctx, [lo], [hi])
        assert ms > 0 and t["wg_per_cu"] in (0, 1, 2)
        plan = sv_mod.sieve_plan(lo, hi, tuning=t)
        if t["bucket_limit"] not in (0, 0xFFFFFFFF):
            assert t["bucket_limit"] in (2 * plan["seg_bits"], 4 * plan["seg_bits"])
        assert gpu.tuning() == t
        assert gpu.count(lo, hi) == oracle_mod.count(lo, hi)
        words, pi = gpu.bitmap(lo, lo + 3 * 10**7 + 11)
        assert pi == oracle_mod.count(lo, lo + 3 * 10**7 + 11)
    finally:
        gpu.tuning(seg_bits=0, dense_limit=0, block_threads=0, wg_per_cu=0, bucket_limit=0)


# -- large-prime hit buckets ---------------------------------------------------

@pytest.mark.parametrize("lo,hi,seg_bits,limit,depth", [
    (10**12, 10**12 + 5 * 10**7, 65536, 65536, 0),       # forced buckets, auto depth
    (10**12 + 1, 10**12 + 3 * 10**7 + 7, 65536, 131072, 0),
    (10**12, 10**12 + 2 * 10**7, 65536, 65536, 64),      # tiny depth: overflow, retry
    (10**13 - 3, 10**13 + 2 * 10**7, 131072, 0, 0),      # automatic choice
    (10**15 - 2**31, 10**15, 0, 0, 0),                   # automatic at the top of the domain
    # segments that are not a power of two: the fill divides offsets by them
    (10**12 + 7, 10**12 + 6 * 10**7 + 3, 622592, 622592, 0),
    (10**13 + 1, 10**13 + 3 * 10**7, 491520, 491520, 0),
    (10**12, 10**12 + 2 * 10**7, 622592, 622592, 64),    # tiny depth: overflow, retry
    # automatic, just past the threshold (sqrt(hi) of two widest segments)
    (1_600_000_000_001, 1_600_000_000_001 + 2**31, 0, 0, 0),
])
def test_bucketed_ranges(gpu, oracle_mod, sv_mod, lo, hi, seg_bits, limit, depth):
    gpu.tuning(seg_bits=seg_bits, bucket_limit=limit, bucket_depth=depth)
    try:
        plan = sv_mod.sieve_plan(lo, hi, tuning=gpu.tuning())
        if limit or hi >= 10**15:
            assert plan["bucket_limit"] > 0
        if not seg_bits and lo == 1_600_000_000_001:
            assert plan["bucket_limit"] == plan["seg_bits"] == 622592
        _cmp_bitmap(gpu, oracle_mod, lo, hi)
    finally:
        gpu.tuning(seg_bits=0, bucket_limit=0, bucket_depth=0)


def test_buckets_off_and_on_agree(gpu, sv_mod, oracle_mod):
    # the same range with the large primes scanned per segment and through
    # hit buckets: both equal the oracle
    lo, hi = 10**14, 10**14 + 6 * 10**7
    gpu.tuning(bucket_limit=0xFFFFFFFF)
    try:
        assert sv_mod.sieve_plan(lo, hi, tuning=gpu.tuning())["bucket_limit"] == 0
        w0, p0 = gpu.bitmap(lo, hi)
        a = w0.cpu().numpy()
    finally:
        gpu.tuning(bucket_limit=0)
    gpu.tuning(bucket_limit=1)  # forced: every prime above the segment size
    try:
        assert sv_mod.sieve_plan(lo, hi, tuning=gpu.tuning())["bucket_limit"] > 0
        w1, p1 = gpu.bitmap(lo, hi)
    finally:
        gpu.tuning(bucket_limit=0)
    assert p0 == p1 and np.array_equal(a, w1.cpu().numpy())
    ref, ref_pi = oracle_mod.bitmap(lo, hi)
    assert p0 == ref_pi and np.array_equal(a.view(np.uint32), ref)


# -- kernel timing switch and the count call's early return ---------------------

def test_timing_is_off_by_default_and_switches(gpu, oracle_mod, sv_mod):
    import torch

    print("case timing switch", flush=True)
    s = sv_mod.Sieve(0)
    try:
        assert s.count(2, 10**6) == 78498
        with pytest.raises(sv_mod.SieveError) as e:
            sv_mod.sieve_last_kernel_ms(s.ctx)  # never timed
        assert e.value.status == sv_mod.sieve.SIEVE_EINVAL
        sv_mod.sieve_set_timing(s.ctx, True)
        assert s.count(2, 10**8) == 5761455
        assert sv_mod.sieve_last_kernel_ms(s.ctx) > 0
        words, pi = s.bitmap(10**9, 10**9 + 10**7)
        assert pi == oracle_mod.count(10**9, 10**9 + 10**7)
        assert sv_mod.sieve_last_kernel_ms(s.ctx) > 0
        pis = s.batch(np.array([10**6, 10**10], dtype=np.uint64), np.array([10**6 + 99991, 10**10 + 10**6],
                                                                           dtype=np.uint64))
        assert int(pis[0]) == oracle_mod.count(10**6, 10**6 + 99991)
        assert sv_mod.sieve_last_kernel_ms(s.ctx) > 0
        n = torch.tensor([97, 91, 2**61 - 1], dtype=torch.int64, device="cuda:0")
        out = torch.empty(3, dtype=torch.uint8, device="cuda:0")
        sv_mod.sieve_is_prime_batch(s.ctx, n, 3, out)
        torch.cuda.synchronize()
        assert out.cpu().tolist() == [1, 0, 1]
        assert sv_mod.sieve_last_kernel_ms(s.ctx) > 0
        sv_mod.sieve_set_timing(s.ctx, False)
        with pytest.raises(sv_mod.SieveError):
            sv_mod.sieve_last_kernel_ms(s.ctx)  # forgotten when turned off
        assert s.count(2, 10**7) == 664579
        with pytest.raises(sv_mod.SieveError):
            sv_mod.sieve_last_kernel_ms(s.ctx)
        # the autotuner times its candidates and leaves timing as it found it
        sv_mod.sieve_autotune(s.ctx, [10**8], [10**8 + 10**7], apply=False)
        with pytest.raises(sv_mod.SieveError):
            sv_mod.sieve_last_kernel_ms(s.ctx)
    finally:
        s.close()


def test_count_calls_back_to_back_on_one_stream(gpu, oracle_mod, sv_mod):
    # count calls return on the published count without synchronising the
    # stream; a run of them on one stream, of every length from a single
    # segment to thousands, with bitmap calls between, must each be exact
    import torch

    print("case back-to-back counts", flush=True)
    stream = torch.cuda.Stream(0)
    rng = random.Random(5)
    cases = [(2, 10**10), (0, 3), (10**12, 10**12 + 64), (7, 10**9)]
    cases += [(a, a + rng.randrange(1, 10**rng.randrange(2, 9))) for a in
              (rng.randrange(0, 10**rng.randrange(3, 14)) for _ in range(40))]
    words = torch.empty(sv_mod.sieve_bitmap_words(0, 10**6), dtype=torch.int32, device="cuda:0")
    for i, (lo, hi) in enumerate(cases):
        pi = sv_mod.sieve_range_count(gpu.ctx, lo, hi, stream=stream)
        assert pi == oracle_mod.count(lo, hi), (lo, hi)
        if i % 5 == 0:
            p2 = sv_mod.sieve_range_bitmap(gpu.ctx, 0, 10**6, words, words.numel(), True, stream=stream)
            assert p2 == 78498
    stream.synchronize()
