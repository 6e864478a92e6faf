"""CPU checks of the segment kernel's work maps: the dense phase's
assignment of primes to (wave, lane) in each of its orders covers every dense
prime exactly once, and the per-wave count of primes it marks (cnt) equals
the lanes that hold one; the shared sparse units cover the uncarried primes
exactly once.  The maps restate the index arithmetic of seg_dense (prime
r0 + lane * nw + wave, r0 stepping by 64 * nw, waves numbered from either
end, inside runs only the first eight waves) and of seg_sparse_shared (unit
w: primes i_begin + 64 w + lane)."""
import pytest


OLDEST_WAVES = 8  # kDenseOldestWaves


def dense_map(n_dense, threads, reversed_order, oldest=False):
    nw_all = threads // 64
    nw = nw_all
    if oldest and nw_all >= OLDEST_WAVES:
        nw = OLDEST_WAVES
    seen = []
    for t_wave in range(nw_all):
        if oldest and nw_all >= OLDEST_WAVES and t_wave >= OLDEST_WAVES:
            continue  # waves 8.. take no dense primes
        wave = nw - 1 - t_wave if (reversed_order or oldest) else t_wave
        r0 = 0
        while r0 + wave < n_dense:
            held = [r0 + lane * nw + wave for lane in range(64) if r0 + lane * nw + wave < n_dense]
            cnt = min(64, (n_dense - r0 - wave + nw - 1) // nw)
            assert cnt == len(held), (n_dense, threads, t_wave, r0)
            # the wave marks the primes of lanes 0..cnt-1, which are exactly those held
            assert held == [r0 + lane * nw + wave for lane in range(cnt)]
            seen += held
            r0 += 64 * nw
    return seen


@pytest.mark.parametrize("threads", [256, 512, 1024])
@pytest.mark.parametrize("n_dense", [0, 1, 15, 16, 63, 64, 65, 187, 1000, 1024, 1025, 5000])
@pytest.mark.parametrize("order", ["plain", "reversed", "oldest"])
def test_dense_map_covers_each_prime_once(threads, n_dense, order):
    seen = dense_map(n_dense, threads, order == "reversed", oldest=order == "oldest")
    assert sorted(seen) == list(range(n_dense))


def test_oldest_order_leaves_the_last_waves_free():
    # inside runs of a 1024-thread workgroup the dense primes go to waves 0..7
    # only, the heaviest share to wave 7; waves 8..15 hold none
    n_dense, threads = 187, 1024
    held = {}
    for t_wave in range(threads // 64):
        if t_wave >= OLDEST_WAVES:
            held[t_wave] = []
            continue
        wave = OLDEST_WAVES - 1 - t_wave
        held[t_wave] = [r0 + lane * OLDEST_WAVES + wave
                        for r0 in range(0, n_dense, 64 * OLDEST_WAVES) for lane in range(64)
                        if r0 + lane * OLDEST_WAVES + wave < n_dense]
    assert all(not held[w] for w in range(8, 16))
    assert held[7][0] == 0  # prime index 0, the smallest dense prime
    assert sum(len(v) for v in held.values()) == n_dense


def shared_units(i_begin, n_primes):
    """Prime indices of each unit of seg_sparse_shared, lane by lane."""
    n_units = (n_primes - i_begin + 63) // 64 if n_primes > i_begin else 0
    return [[i_begin + w * 64 + lane for lane in range(64) if i_begin + w * 64 + lane < n_primes]
            for w in range(n_units)]


@pytest.mark.parametrize("i_begin,n_primes", [(0, 0), (10, 10), (10, 9), (187, 188), (187, 251),
                                              (187, 252), (4283, 9591), (4283, 78497)])
def test_shared_units_cover_the_uncarried_primes_once(i_begin, n_primes):
    units = shared_units(i_begin, n_primes)
    flat = [i for u in units for i in u]
    assert flat == list(range(i_begin, max(i_begin, n_primes)))
    assert all(0 < len(u) <= 64 for u in units)


def test_reversed_order_moves_the_heaviest_share_to_the_last_wave():
    # with the primes ascending (work falling), the plain order gives wave 0
    # the smallest prime of every group of nw, the reversed order the last wave
    n_dense, threads = 187, 1024
    for rev, heavy_wave in ((False, 0), (True, 15)):
        nw = threads // 64
        first = {}
        for t_wave in range(nw):
            wave = nw - 1 - t_wave if rev else t_wave
            first[t_wave] = wave  # lane 0 of this wave holds prime `wave`
        assert min(first, key=first.get) == heavy_wave
