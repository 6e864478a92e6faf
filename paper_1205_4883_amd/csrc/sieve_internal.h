// Internal interface between the host runtime (sieve_api.hip) and the
// kernels (sieve_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sv {

// Odd primes 3..31 are removed by the pre-sieve tables (three groups whose
// products are 15015, 7429 and 899); the marking kernels start at the
// eleventh odd prime, 37.
constexpr uint32_t kPresievePrimes = 10;
constexpr uint32_t kFirstMarkedPrime = 37;

// The widest LDS segment, in words: two 1024-thread workgroups with their
// pre-sieve tables, item word and reduction space still fit in a CU's
// 160 KiB (2 x (792 + 19456) x 4 B plus 136 B each), so a CU keeps 32
// wavefronts while each segment holds 622,592 odd integers (19% more than
// 2^19, for less per-segment set-up).  Not a power of two: the bucket fill
// splits hit offsets by it with a division instead of a shift.
constexpr uint32_t kWideSegWords = 19456;
// LDS words taken by the three pre-sieve tables (each is its pattern's
// period plus one pre-sieve run's words, rounded so the segment starts
// 16-byte aligned).
constexpr uint32_t kTableWords = 792;
// The bootstrap kernel sieves the odd integers below 2^16 in one workgroup.
constexpr uint32_t kBootstrapLimit = 65536;
constexpr uint32_t kBootstrapOddPrimes = 6541;  // odd primes below 2^16

// Work counters and partial counts of one launch.  Device-scope atomics on
// one address serialise across the chip (measured at about 12 ns apiece on
// MI355X, enough to bound a whole launch when every wave adds its count per
// segment), so a launch spreads them over kQueues work counters and kQueues
// count lines, each alone in a 256-byte line, plus one grid word:
//   queue q (uint32_t) at word q * kLineWords,
//   count line q (uint64_t: count << 16 | workgroups added) at word
//     (kQueues + q) * kLineWords,
//   grid word (uint64_t: count << 8 | lines completed) at word kDoneWord.
// Work queue q hands out the items k * kQueues + q, k = 0, 1, ...; workgroup
// b starts on queue b mod kQueues and moves on to the next queue when its own
// runs dry, so every item is taken exactly once whatever the grid size, and
// each workgroup makes at most kQueues failed pops before it leaves.
// A range launch leaves its counter block all zero (the grid word keeps the
// running count between the launches of one call): the workgroup that
// completes the grid word resets it and publishes the count.
constexpr uint32_t kQueues = 8;
constexpr uint32_t kLineWords = 64;
constexpr uint32_t kDoneWord = 2 * kQueues * kLineWords;
constexpr uint32_t kCounterWords = (2 * kQueues + 1) * kLineWords;

// One range as the segment kernels see it.
struct RangeArgs {
    uint64_t first_odd;  // the odd integer of bit 0: (lo & ~1) + 1
    uint64_t nbits;      // odd integers in the range
    uint64_t n_words;    // ceil(nbits / 32)
    uint32_t *out;       // bitmap words of the range (word 0 = bit 0), or null
    uint32_t *counters;  // kCounterWords words, all zero at launch
    bool count;          // count the 1 bits (primes)
    bool last;           // the call's last launch: publish the count and clear it
    unsigned long long *publish;  // where the last launch stores the count (host-mapped or device), or null
    // Large-prime hit buckets of this launch's segments, or null: segment s
    // owns buckets[s * bucket_depth ..) with min(bucket_count[s], depth)
    // entries, each a bit offset inside the segment.
    const uint32_t *buckets;
    const uint32_t *bucket_count;
    uint32_t bucket_depth;
    uint32_t publish_add;  // added to the published count (the even prime 2, when in range)
};

// The marking primes of one launch: odd primes >= 37, ascending.
struct PrimeArgs {
    const uint32_t *primes;
    const double *inv;  // inv[i] = 1 / primes[i], rounded to double
    uint32_t n_dense;   // primes[0, n_dense) are marked a wavefront per prime
    uint32_t n_primes;  // primes[0, n_primes) are used
};

// One interval of a batch, as staged for the device.
struct BatchInterval {
    uint64_t first_odd;
    uint64_t nbits;
    uint64_t n_words;
    uint64_t word_offset;   // into the batch bitmap, or ~0 for count only
    uint32_t n_primes;      // marking primes this interval needs
    uint32_t n_dense;
    uint32_t seg_begin;     // first work item of this interval
    uint32_t pad;
};

// Sizes of a batch launch, in device memory.  The header starts one blob,
// staged in pinned host memory and copied to the device by the batch's stage
// kernel: the interval table sits at byte iv_off and the work list (interval
// index of each item) at item_off.  The blob's second part, kCounterWords
// words at byte kBlobAlign, holds the batch's work queues (zeroed by the
// stage kernel; the count lines are unused).
struct BatchHeader {
    uint32_t n_intervals;
    uint32_t n_items;
    uint32_t seg_words;  // words per work item (segment)
    uint32_t blob_chunks;  // 16-byte chunks of the whole blob (what the stage kernel copies)
    uint64_t iv_off;
    uint64_t item_off;
};
constexpr uint64_t kBlobAlign = 256;
constexpr uint64_t kBlobCounterOff = kBlobAlign;
constexpr uint64_t kBlobIntervalOff = kBlobCounterOff + kCounterWords * 4;

// Launchers (sieve_kernels.hip).  All return the first HIP error.
hipError_t launch_bootstrap_primes(uint32_t *d_out, uint32_t *d_count, hipStream_t s);

// Grid: min(n_segments, max_blocks) workgroups draining the work queues.
// The work items are runs of consecutive segments (range_chunks: n_chunks
// runs of `chunk` segments, then the remaining segments one by one).
constexpr uint32_t kMaxChunk = 8;
void range_chunks(uint32_t n_segments, uint32_t grid, uint32_t *chunk, uint32_t *n_chunks);
hipError_t launch_range(const RangeArgs &r, const PrimeArgs &p, uint32_t seg_words,
                        uint32_t block_threads, uint32_t n_segments, uint32_t max_blocks,
                        hipStream_t s);

// Bucket fill: the hits of primes[0, n_large) (all >= the segment size) on
// the n_segs segments of seg_bits bits (a multiple of 32, at most 622,592)
// starting at the odd integer
// first_odd, in chunks of kBucketChunk segments.  Appends bit offsets to
// buckets[s * depth ..), counting in bucket_count[s] (zero at launch); sets
// *overflow when a segment needs more than depth entries.
constexpr uint32_t kBucketChunk = 32;
hipError_t launch_bucket_fill(const uint32_t *primes, const double *inv, uint32_t n_large,
                              uint64_t first_odd, uint32_t seg_bits, uint32_t n_segs, uint32_t *buckets,
                              uint32_t *bucket_count, uint32_t depth, uint32_t *overflow, hipStream_t s);

// inv[i] = 1.0 / primes[i] for i < n.
hipError_t launch_reciprocals(const uint32_t *d_primes, uint32_t n, double *d_inv, hipStream_t s);

// dst[0, n_words) = src[0, n_words) by a kernel on s; both 16-byte aligned,
// dst may be host memory mapped into the device.
hipError_t launch_copy_words(const uint32_t *src, uint32_t *dst, uint64_t n_words, hipStream_t s);

// Compaction of a bitmap (1 = prime) into the ascending list of the integers
// its set bits stand for.  d_tmp needs compact_tmp_words(n_words) words.
uint64_t compact_tmp_words(uint64_t n_words);
hipError_t launch_compact(const uint32_t *d_words, uint64_t n_words, uint64_t first_odd,
                          uint32_t *d_tmp, uint32_t *d_out, uint32_t *d_total, hipStream_t s);

// Stage kernel (copies the blob from h_blob, the device-visible address of
// its pinned host staging, into d_blob and clears the work queues), the
// persistent batch kernel (each work item's count into item_counts[item])
// and the reduction kernel (counts[k] = the sum over interval k's items;
// counts may be mapped host memory).  All read their sizes and the table
// offsets from the blob's header, so one captured graph serves every batch
// that fits its buffers.  max_intervals sizes the reduction grid.  small:
// every marking prime of the batch is below 2^24 (24-bit products).
constexpr uint32_t kStageBlocks = 64;
hipError_t launch_batch(const void *h_blob, BatchHeader *d_blob, uint32_t max_intervals, const uint32_t *d_primes,
                        const double *d_inv, uint32_t *d_words, uint32_t *d_item_counts,
                        unsigned long long *counts, uint32_t seg_words, uint32_t block_threads,
                        uint32_t n_blocks, bool small, hipStream_t s);

// The segment kernels are built for a few static LDS sizes: the smallest
// capacity (in words) that holds seg_words (0 if none), the LDS bytes a
// workgroup then uses, and the largest segment supported.
uint32_t seg_capacity_for(uint32_t seg_words);
uint32_t lds_bytes_for(uint32_t seg_words);
uint32_t max_seg_words();

// Workgroups of the range / batch kernel that fit on one CU at once (the HIP
// occupancy calculator: LDS, VGPR and SGPR limits).
uint32_t range_blocks_per_cu(uint32_t seg_words, uint32_t threads, bool write);
uint32_t batch_blocks_per_cu(uint32_t seg_words, uint32_t threads);

}  // namespace sv
