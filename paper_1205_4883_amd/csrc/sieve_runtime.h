// Host runtime internals shared by the C ABI (sieve_api.hip) and the serving
// loop (sieve_serve.hip).  Not part of the public ABI.
#pragma once

#include <algorithm>
#include <map>
#include <tuple>
#include <vector>

#include "sieve.h"
#include "sieve_internal.h"

namespace sv {

constexpr uint64_t kMaxPrimeLimit = 31622777;      // > isqrt(SIEVE_MAX_HI)
constexpr uint64_t kDefaultPrimeLimit = 1u << 20;  // covers hi <= 1.0995e12
constexpr uint32_t kSegGranuleWords = 128;         // 4096 bits
constexpr uint32_t kDefaultMaxSegWords = 16384;    // 2^19 bits = 64 KiB of LDS
constexpr uint64_t kDefaultBudget = 32ull << 30;
constexpr uint64_t kBucketPoolBytes = 256ull << 20;  // bucket memory per window of segments
constexpr uint32_t kPiIndexShift = 8;                // block width of the prime-count index

struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

struct HostBuf {  // pinned, coherent host memory, mapped into the device
    void *p = nullptr;
    void *d = nullptr;  // its device-visible address
    size_t bytes = 0;
};

// Everything a captured batch graph bakes in.
struct GraphKey {
    const void *h_blob, *blob, *counts, *item_counts, *primes, *inv;
    uint32_t *words;
    uint32_t seg_words, threads, blocks, max_intervals;
    bool small;  // every marking prime below 2^24
    bool operator==(const GraphKey &o) const
    {
        return h_blob == o.h_blob && blob == o.blob && counts == o.counts && item_counts == o.item_counts &&
               primes == o.primes && inv == o.inv && words == o.words && seg_words == o.seg_words &&
               threads == o.threads && blocks == o.blocks && max_intervals == o.max_intervals && small == o.small;
    }
};

// One batch in flight: the interval table and work list (pinned staging and
// device copies), per-item counts, the per-interval counts (written by the
// device straight into mapped host memory), the batch header and the
// captured graph that launches it.  A context owns one; the server owns one
// per lane.
struct BatchEngine {
    DevBuf blob, item_counts;  // blob: header, work queues, interval table, work list
    HostBuf s_blob, s_counts;
    uint64_t blob_used = 0;  // bytes of the staged blob
    std::vector<uint32_t> order;  // intervals in queue order
    std::vector<uint32_t> nmark;
    std::vector<uint64_t> bound;  // isqrt(hi - 1) per interval
    // one captured graph per variant of the marking kernel: [1] for batches
    // whose marking primes are all below 2^24 (24-bit products), [0] else,
    // so that batches alternating between the two never re-capture
    hipGraph_t graph[2] = {};
    hipGraphExec_t exec[2] = {};
    GraphKey key[2] = {};
    uint64_t captures = 0;  // graphs captured and instantiated so far
    hipEvent_t done = nullptr;  // recorded after the last launch
    bool pending = false;       // a launch has been recorded on `done`
    uint32_t n = 0;             // intervals staged
    uint64_t items = 0;         // work items staged
    uint32_t seg_words = 0, dense_limit = 0, threads = 0;
    bool small = true;  // every marking prime of the staged batch below 2^24
};

}  // namespace sv

struct sieve_ctx {
    int device = 0;
    uint32_t n_cu = 0;
    uint32_t lds_max = 0;  // LDS bytes one workgroup may use
    uint32_t lds_per_cu = 0;
    uint64_t hbm_budget = sv::kDefaultBudget;
    hipStream_t stream = nullptr;
    sieve_tuning tuning{};
    int last_hip = 0;

    // base primes: all odd primes <= primes_limit, ascending
    uint64_t primes_limit = 0;
    std::vector<uint32_t> h_primes;
    std::vector<double> h_recip_prefix;  // sum of 1/p over h_primes[0, i)
    std::vector<uint32_t> h_pi_index;     // [k]: primes in h_primes below k << kPiIndexShift
    uint32_t *d_primes = nullptr;
    double *d_inv = nullptr;  // d_inv[i] = 1 / d_primes[i]

    // Per-call device counters (work queues and partial counts, kCounterWords
    // words each): kSlots slots, the first free one in turn, each guarded by
    // an event so that an asynchronous call still running on another stream
    // never sees its slot reset.  32 covers a server's three lanes with eight
    // plain launches each in flight, so the dispatcher does not wait for one.
    static constexpr int kSlots = 32;
    uint32_t *d_ctr = nullptr;  // kSlots * kCounterWords words
    hipEvent_t slot_done[kSlots] = {};
    bool slot_used[kSlots] = {};
    bool slot_dirty[kSlots] = {};  // not known to be all zero
    int next_slot = 0;
    // pinned and mapped, 64 words: the published count (words 0-1, written
    // by the kernel through d_pub) and the bucket overflow flag (word 16)
    uint32_t *h_ctr = nullptr;
    unsigned long long *d_pub = nullptr;

    // events bracketing the last sieve kernel launch (range, batch or
    // primality), recorded only while timing is on (two event records cost
    // a few microseconds per call)
    hipEvent_t ev_start = nullptr, ev_stop = nullptr;
    bool ev_valid = false;
    bool timing = false;

    sv::BatchEngine batch;

    // large-prime hit buckets of the plain path (grown on demand)
    sv::DevBuf b_buckets, b_bcount;

    // autotuner cache: (batch?, decade of max hi, log2 of total words)
    std::map<std::tuple<int, int, int>, std::pair<sieve_tuning, double>> tune_cache;
};

namespace sv {

#define SV_HIP_TRY(ctx, expr)                       \
    do {                                            \
        hipError_t e_ = (expr);                     \
        if (e_ != hipSuccess) {                     \
            (ctx)->last_hip = static_cast<int>(e_); \
            return SIEVE_EDEVICE;                   \
        }                                           \
    } while (0)

uint64_t isqrt_u64(uint64_t n);
int make_plan(uint64_t lo, uint64_t hi, const sieve_tuning *tu, uint32_t n_cu, uint32_t lds_bytes,
              sieve_plan_info *out);
int ensure_primes(sieve_ctx *c, uint64_t bound);
// Workgroups of the plain range kernel resident on the whole device for a plan.
uint32_t resident_blocks(const sieve_ctx *c, const sieve_plan_info &pl, bool write);
// Once per device, with the context's device current: find the device
// address of the allocation-free call's counter array and clear it
// (sieve_noalloc.hip).
int noalloc_setup(sieve_ctx *c);
void marking_primes(const sieve_ctx *c, uint64_t r, uint32_t dense_limit, uint32_t *n_mark,
                    uint32_t *n_dense);
// The plain path: sieve [lo, hi) into d_words (may be null) and/or count it.
int run_range(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, uint64_t *pi_out,
              hipStream_t s);
// The plain path enqueued without waiting, for a caller that tracks
// completion itself: the launch publishes the count of odd primes (2 not
// included) to *d_pub, a device-visible pinned word.  Returns kNotAsync,
// enqueueing nothing, when the range is empty or needs hit buckets (whose
// overflow check needs a host round trip).
constexpr int kNotAsync = 1;
int range_async(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, unsigned long long *d_pub,
                hipStream_t s);
// Whether range_async would enqueue [lo, hi) (a valid, non-empty range that
// needs no hit buckets).
bool range_async_ok(const sieve_ctx *c, uint64_t lo, uint64_t hi);
int grow(sieve_ctx *c, DevBuf &b, size_t bytes);
int grow_host(sieve_ctx *c, HostBuf &b, size_t bytes);

// Batch engine.  stage: validate the intervals and build the work list in
// the engine's pinned staging (waits for the engine's previous launch).
// launch: launch the batch graph on s (asynchronous; its first kernel copies
// the staging to the device); the counts (excluding the even prime 2) land
// in counts_host() once `done` completes.
int engine_init(sieve_ctx *c, BatchEngine &e);
// Grow the engine's buffers ahead of time for n intervals and `items` work
// items, so that batches up to that size never re-capture the graph.
int engine_reserve(sieve_ctx *c, BatchEngine &e, uint32_t n, uint64_t items);
void engine_free(BatchEngine &e);
int engine_stage(sieve_ctx *c, BatchEngine &e, const sieve_interval *iv, uint32_t n, uint32_t *d_words,
                 uint64_t total_words);
int engine_launch(sieve_ctx *c, BatchEngine &e, uint32_t *d_words, hipStream_t s, bool timed);
// Capture (if not yet captured for the engine's current buffers and tuning)
// the graph variant `small` of a batch writing into d_words; runs nothing.
// Lets a caller capture both variants ahead of time, after a first stage.
int engine_graph(sieve_ctx *c, BatchEngine &e, uint32_t *d_words, bool small);
// Words per work item (segment) of a batch on this context's tuning.
uint32_t batch_seg_words(const sieve_ctx *c);
// Bytes engine_reserve(n, items) holds on the device.
uint64_t engine_device_bytes(uint32_t n, uint64_t items);
hipError_t launch_is_prime(const uint64_t *d_n, uint64_t count, uint8_t *d_out, uint32_t blocks, hipStream_t s);
hipError_t launch_fermat(const uint64_t *d_n, uint64_t count, const uint64_t *d_draws, uint32_t iterations,
                         uint8_t *d_out, uint32_t blocks, hipStream_t s);

inline const unsigned long long *counts_host(const BatchEngine &e)
{
    return static_cast<const unsigned long long *>(e.s_counts.p);
}

}  // namespace sv
