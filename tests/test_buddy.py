"""CPU tests of the serving loop's buddy allocator (csrc/buddy.h), which
hands out the device bitmap pool and the pinned host arena: blocks never
overlap, stay inside the region and aligned to their size, every byte of the
region is usable, and freeing everything merges the region back into its
root blocks.  A small C++ driver is compiled with g++ and replays a seeded
random sequence of allocations and frees."""
import os
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_1205_4883_amd", "csrc")

DRIVER = r"""
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>
#include "buddy.h"

struct Blk { uint64_t off; int order; };

static int fail(const char *what) { std::printf("FAIL %s\n", what); return 1; }

int main(int argc, char **argv)
{
    const uint64_t bytes = std::strtoull(argv[1], nullptr, 10);
    const uint64_t max_block = std::strtoull(argv[2], nullptr, 10);
    sv::Buddy b;
    const uint64_t size = b.init(bytes, max_block);
    // every byte of the region, rounded down to 4 KiB, is usable
    if (size != (bytes >> 12 << 12)) return fail("size");
    if (b.max_block() > max_block * 2 - 1 && max_block >= 4096) return fail("max_block");
    std::mt19937_64 rng(12345);
    std::vector<Blk> live;
    std::vector<unsigned char> owner(size >> 12, 0);
    for (int step = 0; step < 200000; ++step) {
        const bool do_alloc = live.empty() || (rng() % 100) < 55;
        if (do_alloc) {
            const uint64_t want = 1 + rng() % (b.max_block() ? b.max_block() : 4096);
            Blk k;
            if (!b.alloc(want, &k.off, &k.order)) continue;
            const uint64_t len = uint64_t(1) << k.order;
            if (len < want) return fail("short block");
            if (k.off % len) return fail("misaligned");
            if (k.off + len > size) return fail("outside");
            for (uint64_t p = k.off >> 12; p < (k.off + len) >> 12; ++p) {
                if (owner[p]) return fail("overlap");
                owner[p] = 1;
            }
            live.push_back(k);
        } else {
            const size_t i = rng() % live.size();
            const Blk k = live[i];
            live[i] = live.back();
            live.pop_back();
            for (uint64_t p = k.off >> 12; p < (k.off + (uint64_t(1) << k.order)) >> 12; ++p) owner[p] = 0;
            b.free(k.off, k.order);
        }
        uint64_t used = 0;
        for (const Blk &k : live) used += uint64_t(1) << k.order;
        if (used != b.used()) return fail("used");
    }
    for (const Blk &k : live) b.free(k.off, k.order);
    if (b.used() != 0) return fail("used at end");
    // after every free the whole region is back: the largest block fits as
    // many times as the root blocks of that size allow
    std::vector<Blk> again;
    Blk k;
    const uint64_t top = b.max_block();
    uint64_t n_top = 0;
    while (top && b.alloc(top, &k.off, &k.order)) { again.push_back(k); ++n_top; }
    if (top && n_top != size / top) return fail("merge to the largest blocks");
    for (const Blk &x : again) b.free(x.off, x.order);
    again.clear();
    while (b.alloc(4096, &k.off, &k.order)) again.push_back(k);
    if (again.size() != (size >> 12)) return fail("every 4 KiB block");
    std::printf("OK %llu\n", (unsigned long long)size);
    return 0;
}
"""


@pytest.fixture(scope="module")
def driver(tmp_path_factory):
    d = tmp_path_factory.mktemp("buddy")
    src = d / "buddy_driver.cpp"
    src.write_text(DRIVER)
    exe = d / "buddy_driver"
    subprocess.run(["g++", "-O2", "-std=c++17", "-I", CSRC, str(src), "-o", str(exe)], check=True)
    return str(exe)


@pytest.mark.parametrize("bytes_,max_block", [
    (1 << 24, 1 << 20),                # whole root blocks
    ((1 << 24) + (5 << 12), 1 << 20),  # plus the binary digits of the rest
    (3 << 20, 1 << 22),                # max block above the region
    (4096, 1 << 20),                   # one minimum block
    (100 * (1 << 20) + 12345, 1 << 23),
])
def test_buddy_allocator(driver, bytes_, max_block):
    r = subprocess.run([driver, str(bytes_), str(max_block)], capture_output=True, text=True)
    assert r.returncode == 0 and r.stdout.startswith("OK"), r.stdout + r.stderr
