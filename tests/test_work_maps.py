"""CPU checks of the segment kernel's work maps: the dense phase's
assignment of primes to (wave, lane) in either wave order covers every dense
prime exactly once, and the per-wave count of primes it marks (cnt) equals
the lanes that hold one.  The maps restate the index arithmetic of seg_dense
(prime r0 + lane * nw + wave, r0 stepping by 64 * nw, waves numbered from
either end)."""
import pytest


def dense_map(n_dense, threads, reversed_order):
    nw = threads // 64
    seen = []
    for t_wave in range(nw):
        wave = nw - 1 - t_wave if reversed_order else t_wave
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
@pytest.mark.parametrize("reversed_order", [False, True])
def test_dense_map_covers_each_prime_once(threads, n_dense, reversed_order):
    seen = dense_map(n_dense, threads, reversed_order)
    assert sorted(seen) == list(range(n_dense))


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
