// Serving loop with continuous batching (declared in sieve.h).
//
// One dispatcher thread owns the server's context.  Submitted requests wait
// in arrival order until their bitmap gets a block of the device pool (the
// HBM budget less the server's fixed device memory, allocated once at
// creation) and a block of the pinned host arena (admission).  Whenever a
// lane (a stream with its own batch engine) is free, the dispatcher packs the
// admitted requests into one batch, launches its graph (captured at
// creation), queues the bitmap copies to the requests' host blocks, and
// records an event; lanes finish independently, so batches overlap on the
// device while new arrivals form the next batch.  The plain mode serves one
// request at a time with the plain range launch, for comparison.
#include <algorithm>
#include <atomic>
#include <chrono>
#include <condition_variable>
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <iterator>
#include <map>
#include <mutex>
#include <new>
#include <set>
#include <thread>
#include <unordered_map>
#include <vector>

#include "buddy.h"
#include "sieve_runtime.h"

namespace {

uint64_t now_ns()
{
    return static_cast<uint64_t>(std::chrono::duration_cast<std::chrono::nanoseconds>(
                                     std::chrono::steady_clock::now().time_since_epoch())
                                     .count());
}

struct Request {
    uint64_t id = 0, lo = 0, hi = 0, n_words = 0;
    uint32_t flags = 0;
    uint64_t items = 0;  // batch work items (segments)
    uint64_t t_submit = 0, t_admit = 0, t_launch = 0, t_done = 0;
    uint64_t pi = 0;
    int status = SIEVE_OK;
    // a bitmap request holds a device block (its words, from admission until
    // the copy to the host is done) and a pinned host block (until released)
    uint64_t dev_off = 0, host_off = 0;
    int dev_order = -1, host_order = -1;
    uint32_t *host = nullptr;
};

struct Lane {
    hipStream_t stream = nullptr;
    sv::BatchEngine eng;
    hipEvent_t copied = nullptr;  // after the bitmap copies
    std::vector<Request *> reqs;
    std::vector<sieve_interval> iv;
    bool busy = false;
    bool single = false;  // the launches in flight are plain range launches, one per request
    uint64_t calls = 0;   // launch calls made on this lane (for the slow-call log)
    uint64_t t_launch = 0;
    // pinned and mapped: the counts plain launches publish, one word per
    // request (kMaxPlainBatch)
    volatile unsigned long long *h_pub = nullptr;
    unsigned long long *d_pub = nullptr;
};

constexpr unsigned long long kUnpublished = ~0ull;
// Batches of up to this many requests go as plain launches, one per request.
constexpr size_t kMaxPlainBatch = 8;

}  // namespace

struct sieve_server {
    sieve_server_config cfg{};
    sieve_ctx *ctx = nullptr;
    std::vector<Lane> lanes;
    // device memory for the bitmaps of admitted requests (the HBM budget
    // less the server's fixed device memory) and pinned host memory for the
    // returned bitmaps
    uint32_t *d_pool = nullptr;
    sv::Buddy pool;
    void *h_arena = nullptr;
    char *d_arena = nullptr;  // the arena's device-visible address
    sv::Buddy arena;
    uint64_t items_cap = 0;        // work items a batch may hold
    uint64_t captures_at_create = 0;
    // Steps of the launch call in progress (dispatcher thread only): with
    // SIEVE_SERVE_LOG_SLOW set in the environment, a call over 1 ms prints
    // how long each of its steps took.
    bool log_slow = false;
    static constexpr int kMaxSteps = 24;  // a call of eight plain launches takes 18
    int n_steps = 0;
    const char *step_name[kMaxSteps] = {};
    uint64_t step_ns[kMaxSteps] = {};

    std::mutex m;
    std::condition_variable cv_work;  // dispatcher: new submissions or stop
    std::condition_variable cv_done;  // pollers: new results
    std::deque<Request *> pending;    // submitted, not admitted
    std::deque<Request *> admitted;   // admitted, waiting for a lane
    std::deque<Request *> done;       // finished, not yet polled
    std::unordered_map<uint64_t, Request *> held;  // polled bitmap results, until release
    uint64_t next_id = 1;
    bool stop = false;
    int fatal = SIEVE_OK;
    sieve_server_stats stats{};
    std::thread worker;
};

namespace {

void step(sieve_server *s, const char *name)
{
    if (s->n_steps < sieve_server::kMaxSteps) {
        s->step_name[s->n_steps] = name;
        s->step_ns[s->n_steps++] = now_ns();
    }
}

constexpr uint32_t kDefaultLanes = 3;
constexpr uint32_t kDefaultMaxBatch = 1024;
constexpr uint64_t kDefaultBatchWords = 1ull << 26;
constexpr uint64_t kDefaultArena = 2ull << 30;
constexpr uint64_t kMinItemsCap = 1ull << 16;
// Device memory of the server's context that the HBM budget is charged with
// before its bitmap pool: the full base-prime table (primes below
// 31,622,777 and their reciprocals, built at creation: 23 MB) with room to
// build it, and the counter slots.  The plain mode adds the hit-bucket pool
// of run_range, the batched mode each lane's batch buffers.
constexpr uint64_t kContextBytes = 64ull << 20;

bool wants_words(const Request *r)
{
    return (r->flags & SIEVE_WANT_BITMAP) && r->n_words;
}

// Admit from the head of the pending queue while a device block and a host
// block can be had for its bitmap (both budgets are real memory: the device
// pool and the pinned arena).  A request that cannot be placed waits, and so
// does everything behind it (arrival order).
void admit_locked(sieve_server *s)
{
    while (!s->pending.empty()) {
        Request *r = s->pending.front();
        if (wants_words(r)) {
            const uint64_t bytes = r->n_words * 4;
            if (!s->pool.alloc(bytes, &r->dev_off, &r->dev_order)) {
                ++s->stats.deferred;
                return;
            }
            if (!s->arena.alloc(bytes, &r->host_off, &r->host_order)) {
                s->pool.free(r->dev_off, r->dev_order);
                r->dev_order = -1;
                ++s->stats.deferred;
                return;
            }
            r->host = reinterpret_cast<uint32_t *>(static_cast<char *>(s->h_arena) + r->host_off);
        }
        s->stats.peak_admitted_bytes = std::max<uint64_t>(s->stats.peak_admitted_bytes, s->pool.used());
        s->stats.peak_host_bytes = std::max<uint64_t>(s->stats.peak_host_bytes, s->arena.used());
        r->t_admit = now_ns();
        s->pending.pop_front();
        s->admitted.push_back(r);
    }
}

uint32_t *dev_words(sieve_server *s, const Request *r)
{
    return wants_words(r) ? s->d_pool + r->dev_off / 4 : nullptr;
}

// The device-visible address of a request's block of the host arena.
uint32_t *arena_words(sieve_server *s, const Request *r)
{
    return reinterpret_cast<uint32_t *>(s->d_arena + r->host_off);
}

// A request is finished: its device block goes back to the pool (its copy
// to the host is complete); the host block stays until released.
void finish_locked(sieve_server *s, Request *r)
{
    if (r->dev_order >= 0) {
        s->pool.free(r->dev_off, r->dev_order);
        r->dev_order = -1;
    }
    r->t_done = now_ns();
    ++s->stats.completed;
    s->done.push_back(r);
}

// Take admitted requests for one batch (under the lock), within the batch's
// request, word and work-item caps (the lane's buffers and graphs are sized
// for them at creation, so a batch never re-captures its graph).
void take_batch_locked(sieve_server *s, Lane &lane)
{
    uint64_t words = 0, items = 0;
    lane.reqs.clear();
    while (!s->admitted.empty() && lane.reqs.size() < s->cfg.max_batch) {
        Request *r = s->admitted.front();
        const uint64_t w = wants_words(r) ? r->n_words : 0;
        if (!lane.reqs.empty() && (words + w > s->cfg.max_batch_words || items + r->items > s->items_cap))
            break;
        words += w;
        items += r->items;
        s->admitted.pop_front();
        lane.reqs.push_back(r);
    }
}

// A small batch (up to kMaxPlainBatch requests) goes as plain range
// launches, one per request, one after another on the lane's stream: no
// batch staging and no graph, the lowest latency when requests arrive a few
// at a time.  Each count is published to the request's pinned word of the
// lane.  Returns sv::kNotAsync, enqueueing nothing, when a range is not
// eligible (empty, or bucketed): the batch then takes the batch launch.
int launch_single_lane(sieve_server *s, Lane &lane)
{
    sieve_ctx *c = s->ctx;
    if (lane.reqs.size() > kMaxPlainBatch)
        return sv::kNotAsync;
    for (const Request *r : lane.reqs)
        if (!sv::range_async_ok(c, r->lo, r->hi))
            return sv::kNotAsync;
    for (size_t j = 0; j < lane.reqs.size(); ++j) {
        Request *r = lane.reqs[j];
        uint32_t *d = dev_words(s, r);
        lane.h_pub[j] = kUnpublished;
        r->t_launch = now_ns();
        const int st = sv::range_async(c, r->lo, r->hi, d, lane.d_pub + j, lane.stream);
        if (st != SIEVE_OK)
            return st == sv::kNotAsync ? SIEVE_EDEVICE : st;  // checked eligible above
        step(s, "range launch");
        if (d)
            SV_HIP_TRY(c, sv::launch_copy_words(d, arena_words(s, r), r->n_words, lane.stream));
        step(s, "bitmap copy");
    }
    SV_HIP_TRY(c, hipEventRecord(lane.copied, lane.stream));
    step(s, "event");
    lane.single = true;
    lane.busy = true;
    return SIEVE_OK;
}

int launch_batch_lane(sieve_server *s, Lane &lane)
{
    sieve_ctx *c = s->ctx;
    const uint32_t n = static_cast<uint32_t>(lane.reqs.size());
    lane.iv.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        const Request *r = lane.reqs[i];
        sieve_interval &v = lane.iv[i];
        v.lo = r->lo;
        v.hi = r->hi;
        v.flags = wants_words(r) ? SIEVE_WANT_BITMAP : 0;
        v.pad = 0;
        v.word_offset = v.flags ? r->dev_off / 4 : 0;  // the request's block of the pool
    }
    if (int st = sv::engine_stage(c, lane.eng, lane.iv.data(), n, s->d_pool, s->pool.size() / 4))
        return st;
    step(s, "batch stage");
    const uint64_t t = now_ns();
    for (Request *r : lane.reqs)
        r->t_launch = t;
    if (int st = sv::engine_launch(c, lane.eng, s->d_pool, lane.stream, false))
        return st;
    step(s, "batch launch");
    for (const Request *r : lane.reqs)
        if (wants_words(r))
            SV_HIP_TRY(c, sv::launch_copy_words(dev_words(s, r), arena_words(s, r), r->n_words, lane.stream));
    step(s, "bitmap copies");
    SV_HIP_TRY(c, hipEventRecord(lane.copied, lane.stream));
    step(s, "event");
    lane.single = false;
    lane.busy = true;
    return SIEVE_OK;
}

// Plain mode: one request, plain range launch, bitmap copy, wait.
int serve_plain(sieve_server *s, Lane &lane, Request *r)
{
    sieve_ctx *c = s->ctx;
    r->t_launch = now_ns();
    uint64_t pi = 0;
    uint32_t *d = dev_words(s, r);
    if (int st = sv::run_range(c, r->lo, r->hi, d, &pi, lane.stream))
        return st;
    if (d) {
        SV_HIP_TRY(c, hipMemcpyAsync(r->host, d, r->n_words * 4, hipMemcpyDeviceToHost, lane.stream));
        SV_HIP_TRY(c, hipStreamSynchronize(lane.stream));
    }
    r->pi = pi;
    return SIEVE_OK;
}

// How long the dispatcher keeps polling after its last activity before it
// blocks on the submission condition variable.
constexpr uint64_t kSpinNs = 200000;

void dispatcher(sieve_server *s)
{
    sieve_ctx *c = s->ctx;
    (void)hipSetDevice(c->device);
    const bool plain = s->cfg.mode == SIEVE_SERVE_PLAIN;
    uint64_t last_active = now_ns();
    for (;;) {
        bool progressed = false;
        // 1. retire finished lanes
        for (Lane &lane : s->lanes) {
            if (!lane.busy || hipEventQuery(lane.copied) != hipSuccess)
                continue;
            std::lock_guard<std::mutex> g(s->m);
            if (lane.single) {
                for (size_t j = 0; j < lane.reqs.size(); ++j) {
                    Request *r = lane.reqs[j];
                    const unsigned long long v = lane.h_pub[j];
                    if (v == kUnpublished)
                        r->status = SIEVE_EDEVICE;
                    r->pi = v + ((r->lo <= 2 && 2 < r->hi) ? 1 : 0);
                    finish_locked(s, r);
                }
            } else {
                lane.eng.pending = false;
                const unsigned long long *cnt = sv::counts_host(lane.eng);
                for (size_t i = 0; i < lane.reqs.size(); ++i) {
                    Request *r = lane.reqs[i];
                    r->pi = cnt[i] + ((r->lo <= 2 && 2 < r->hi) ? 1 : 0);
                    finish_locked(s, r);
                }
            }
            lane.reqs.clear();
            lane.busy = false;
            progressed = true;
            s->cv_done.notify_all();
        }
        // 2. admit and launch on free lanes
        int inflight = 0;
        for (Lane &lane : s->lanes)
            inflight += lane.busy ? 1 : 0;
        for (Lane &lane : s->lanes) {
            if (lane.busy)
                continue;
            {
                std::lock_guard<std::mutex> g(s->m);
                admit_locked(s);
                lane.reqs.clear();
                if (plain) {
                    if (!s->admitted.empty()) {
                        lane.reqs.push_back(s->admitted.front());
                        s->admitted.pop_front();
                    }
                } else {
                    take_batch_locked(s, lane);
                }
            }
            if (lane.reqs.empty())
                break;
            int st;
            if (plain) {
                st = serve_plain(s, lane, lane.reqs[0]);
                std::lock_guard<std::mutex> g(s->m);
                ++s->stats.batches;
                s->stats.max_batch_seen = std::max<uint64_t>(s->stats.max_batch_seen, 1);
                s->stats.max_inflight = std::max<uint64_t>(s->stats.max_inflight, 1);
                lane.reqs[0]->status = st;
                finish_locked(s, lane.reqs[0]);
                lane.reqs.clear();
                s->cv_done.notify_all();
            } else {
                const uint64_t t_call = now_ns();
                s->n_steps = 0;
                step(s, "start");
                st = launch_single_lane(s, lane);
                const bool single = st == SIEVE_OK;
                if (st == sv::kNotAsync)
                    st = launch_batch_lane(s, lane);
                const uint64_t call_ns = now_ns() - t_call;
                ++lane.calls;
                lane.t_launch = t_call;
                std::lock_guard<std::mutex> g(s->m);
                s->stats.max_launch_call_ns = std::max(s->stats.max_launch_call_ns, call_ns);
                s->stats.slow_launch_calls += call_ns > 1000000 ? 1 : 0;
                if (s->log_slow && call_ns > 1000000) {
                    std::fprintf(stderr, "sieve server: lane %d call %llu of %zu request(s) took %.3f ms:",
                                 static_cast<int>(&lane - s->lanes.data()),
                                 static_cast<unsigned long long>(lane.calls), lane.reqs.size(), call_ns * 1e-6);
                    for (int k = 1; k < s->n_steps; ++k)
                        std::fprintf(stderr, " %s %.3f", s->step_name[k],
                                     (s->step_ns[k] - s->step_ns[k - 1]) * 1e-6);
                    // what the other lanes had in flight when this call began
                    for (const Lane &o : s->lanes)
                        if (&o != &lane && o.busy)
                            std::fprintf(stderr, " | lane %d busy %s for %.3f ms (%zu requests)",
                                         static_cast<int>(&o - s->lanes.data()), o.single ? "single" : "batch",
                                         (t_call - o.t_launch) * 1e-6, o.reqs.size());
                    std::fprintf(stderr, "\n");
                }
                ++s->stats.batches;
                s->stats.single_launches += single ? 1 : 0;
                s->stats.max_batch_seen = std::max<uint64_t>(s->stats.max_batch_seen, lane.reqs.size());
                s->stats.max_inflight = std::max<uint64_t>(s->stats.max_inflight, ++inflight);
                if (st != SIEVE_OK) {
                    for (Request *r : lane.reqs) {
                        r->status = st;
                        finish_locked(s, r);
                    }
                    lane.reqs.clear();
                    lane.busy = false;
                    s->fatal = st;
                    s->cv_done.notify_all();
                }
            }
            progressed = true;
        }
        // 3. wait.  While a launch is in flight, or requests wait for a lane
        //    or for budget, or shortly after the last activity, poll again at
        //    once (yielding the core): a timed sleep costs tens of
        //    microseconds of timer slack per wake-up, more than a small
        //    request takes on the device.  Idle for longer: block until a
        //    submission.
        std::unique_lock<std::mutex> lk(s->m);
        bool busy = false;
        for (Lane &lane : s->lanes)
            busy = busy || lane.busy;
        if (s->stop && !busy && s->pending.empty() && s->admitted.empty())
            return;
        const uint64_t t = now_ns();
        if (progressed)
            last_active = t;
        if (!progressed) {
            const bool waiting = !s->pending.empty() || !s->admitted.empty();
            if (busy || waiting || t - last_active < kSpinNs) {
                lk.unlock();
                std::this_thread::yield();
            } else if (!s->stop) {
                s->cv_work.wait_for(lk, std::chrono::milliseconds(5));
                last_active = now_ns();
            }
        }
    }
}

uint64_t total_captures(const sieve_server *s)
{
    uint64_t n = 0;
    for (const Lane &lane : s->lanes)
        n += lane.eng.captures;
    return n;
}

}  // namespace

extern "C" {

int sieve_server_create(int hip_device, const sieve_server_config *cfg, sieve_server **out)
{
    if (!out)
        return SIEVE_EINVAL;
    sieve_server *s = new (std::nothrow) sieve_server();
    if (!s)
        return SIEVE_ENOMEM;
    if (cfg)
        s->cfg = *cfg;
    if (s->cfg.mode > SIEVE_SERVE_PLAIN) {
        delete s;
        return SIEVE_EINVAL;
    }
    if (!s->cfg.lanes)
        s->cfg.lanes = s->cfg.mode == SIEVE_SERVE_PLAIN ? 1 : kDefaultLanes;
    if (!s->cfg.max_batch)
        s->cfg.max_batch = kDefaultMaxBatch;
    if (!s->cfg.max_batch_words)
        s->cfg.max_batch_words = kDefaultBatchWords;
    if (!s->cfg.hbm_budget_bytes)
        s->cfg.hbm_budget_bytes = sv::kDefaultBudget;
    if (!s->cfg.host_arena_bytes)
        s->cfg.host_arena_bytes = kDefaultArena;
    if (s->cfg.lanes > 16 || s->cfg.max_batch_words > (1ull << 32)) {
        delete s;
        return SIEVE_EINVAL;
    }
    s->items_cap = std::max<uint64_t>(kMinItemsCap, 16ull * s->cfg.max_batch);
    s->log_slow = std::getenv("SIEVE_SERVE_LOG_SLOW") != nullptr;
    // The HBM budget is charged with the server's fixed device memory first
    // (the context and each lane's batch buffers); the rest is the bitmap
    // pool, allocated here, so that admitted requests never hold more.
    const bool plain = s->cfg.mode == SIEVE_SERVE_PLAIN;
    const uint64_t fixed = kContextBytes +
                           (plain ? sv::kBucketPoolBytes + (1ull << 20)  // run_range's hit buckets
                                  : s->cfg.lanes * sv::engine_device_bytes(s->cfg.max_batch, s->items_cap));
    if (s->cfg.hbm_budget_bytes < fixed + (1u << sv::Buddy::kMinOrder)) {
        delete s;
        return SIEVE_ENOMEM;
    }
    const uint64_t max_block = s->cfg.max_batch_words * 4;
    int st = sieve_create(&s->ctx, hip_device, s->cfg.hbm_budget_bytes);
    if (st == SIEVE_OK)
        st = sv::ensure_primes(s->ctx, sv::kMaxPrimeLimit);  // no table growth while serving
    if (st == SIEVE_OK) {
        const uint64_t pool = s->pool.init(s->cfg.hbm_budget_bytes - fixed, max_block);
        if (hipMalloc(reinterpret_cast<void **>(&s->d_pool), pool) != hipSuccess) {
            s->d_pool = nullptr;
            st = SIEVE_ENOMEM;
        }
        s->stats.device_pool_bytes = pool;
    }
    if (st == SIEVE_OK) {
        const uint64_t arena = s->arena.init(s->cfg.host_arena_bytes, max_block);
        if (arena == 0 ||
            hipHostMalloc(&s->h_arena, arena, hipHostMallocMapped | hipHostMallocCoherent) != hipSuccess) {
            s->h_arena = nullptr;
            st = SIEVE_ENOMEM;
        } else if (hipHostGetDevicePointer(reinterpret_cast<void **>(&s->d_arena), s->h_arena, 0) != hipSuccess) {
            st = SIEVE_EDEVICE;
        }
        // Copy device memory over the whole arena once, so that the first
        // bitmap copied into each of its blocks while serving does not pay
        // for first-use set-up of its pages.
        const uint64_t pool = s->pool.size();
        for (uint64_t off = 0; st == SIEVE_OK && off < arena; off += pool) {
            const uint64_t n = std::min<uint64_t>(pool, arena - off);
            if (hipMemcpy(static_cast<char *>(s->h_arena) + off, s->d_pool, n, hipMemcpyDeviceToHost) != hipSuccess)
                st = SIEVE_EDEVICE;
        }
    }
    s->lanes.resize(s->cfg.lanes);
    for (Lane &lane : s->lanes) {
        if (st != SIEVE_OK)
            break;
        hipError_t e = hipStreamCreateWithFlags(&lane.stream, hipStreamNonBlocking);
        if (e == hipSuccess)
            e = hipEventCreateWithFlags(&lane.copied, hipEventDisableTiming);
        void *pub = nullptr;
        if (e == hipSuccess)
            e = hipHostMalloc(&pub, kMaxPlainBatch * sizeof(unsigned long long),
                              hipHostMallocMapped | hipHostMallocCoherent);
        if (e == hipSuccess) {
            lane.h_pub = static_cast<volatile unsigned long long *>(pub);
            e = hipHostGetDevicePointer(reinterpret_cast<void **>(&lane.d_pub), pub, 0);
        }
        if (e != hipSuccess)
            st = e == hipErrorOutOfMemory ? SIEVE_ENOMEM : SIEVE_EDEVICE;
        if (st == SIEVE_OK)
            st = sv::engine_init(s->ctx, lane.eng);
        if (plain)
            continue;
        // Size the lane's batch buffers for a full batch and capture both
        // graph variants now: a capture on the dispatcher thread would stall
        // every lane in the middle of serving.
        if (st == SIEVE_OK)
            st = sv::engine_reserve(s->ctx, lane.eng, s->cfg.max_batch, s->items_cap);
        if (st == SIEVE_OK) {
            const sieve_interval none{0, 0, 0, 0, 0};
            st = sv::engine_stage(s->ctx, lane.eng, &none, 1, s->d_pool, s->pool.size() / 4);
        }
        if (st == SIEVE_OK)
            st = sv::engine_graph(s->ctx, lane.eng, s->d_pool, false);
        if (st == SIEVE_OK)
            st = sv::engine_graph(s->ctx, lane.eng, s->d_pool, true);
        // Launch each graph once on the lane's stream with the empty batch:
        // a graph's first launch uploads it to the device, a cost that does
        // not belong in the middle of serving.
        for (int v = 0; v < 2 && st == SIEVE_OK; ++v) {
            lane.eng.small = v == 1;
            st = sv::engine_launch(s->ctx, lane.eng, s->d_pool, lane.stream, false);
            if (st == SIEVE_OK && hipStreamSynchronize(lane.stream) != hipSuccess)
                st = SIEVE_EDEVICE;
            lane.eng.pending = false;
        }
    }
    // Warm every lane before serving: one large bitmap copy to the host on
    // its stream, and one launch of each plain range kernel the loop may use
    // (every segment capacity, counting and writing).  First uses cost
    // milliseconds that would otherwise land on the first requests.
    for (Lane &lane : s->lanes) {
        if (st != SIEVE_OK)
            break;
        const uint64_t copy = std::min<uint64_t>({64ull << 20, s->pool.size(), s->arena.size()});
        if ((plain ? hipMemcpyAsync(s->h_arena, s->d_pool, copy, hipMemcpyDeviceToHost, lane.stream)
                   : sv::launch_copy_words(s->d_pool, reinterpret_cast<uint32_t *>(s->d_arena), copy / 4,
                                           lane.stream)) != hipSuccess)
            st = SIEVE_EDEVICE;
        const uint64_t words_cap = s->pool.size() / 4;
        for (uint64_t n_words : {10000ull, 800000ull, 3000000ull, 8000000ull, 40000000ull}) {
            for (int bm = 0; bm < 2 && st == SIEVE_OK; ++bm) {
                if (bm && n_words > words_cap)
                    continue;
                const int r = sv::range_async(s->ctx, 0, 64 * n_words, bm ? s->d_pool : nullptr, lane.d_pub,
                                              lane.stream);
                if (r != SIEVE_OK && r != sv::kNotAsync)
                    st = r;
            }
        }
        if (st == SIEVE_OK && hipStreamSynchronize(lane.stream) != hipSuccess)
            st = SIEVE_EDEVICE;
    }
    if (st != SIEVE_OK) {
        s->stop = true;
        sieve_server_destroy(s);
        return st;
    }
    s->captures_at_create = total_captures(s);
    s->worker = std::thread(dispatcher, s);
    *out = s;
    return SIEVE_OK;
}

int sieve_server_submit(sieve_server *s, uint64_t lo, uint64_t hi, uint32_t flags, uint64_t *id_out)
{
    if (!s || !id_out || lo > hi)
        return SIEVE_EINVAL;
    if (hi > SIEVE_MAX_HI)
        return SIEVE_ERANGE;
    Request *r = new (std::nothrow) Request();
    if (!r)
        return SIEVE_ENOMEM;
    r->lo = lo;
    r->hi = hi;
    r->flags = flags & SIEVE_WANT_BITMAP;
    r->n_words = sieve_bitmap_words(lo, hi);
    const uint32_t sw = sv::batch_seg_words(s->ctx);
    r->items = (r->n_words + sw - 1) / sw;
    if (wants_words(r) && (r->n_words > s->cfg.max_batch_words || r->n_words * 4 > s->pool.max_block() ||
                           r->n_words * 4 > s->arena.max_block())) {
        delete r;
        return SIEVE_ENOMEM;
    }
    r->t_submit = now_ns();
    {
        std::lock_guard<std::mutex> g(s->m);
        if (s->stop) {
            delete r;
            return SIEVE_EINVAL;
        }
        r->id = s->next_id++;
        *id_out = r->id;
        ++s->stats.submitted;
        s->pending.push_back(r);
    }
    s->cv_work.notify_one();
    return SIEVE_OK;
}

int sieve_server_poll(sieve_server *s, sieve_result *out, uint32_t max, uint32_t *n_out, uint32_t wait_us)
{
    if (!s || !n_out || (max && !out))
        return SIEVE_EINVAL;
    std::unique_lock<std::mutex> lk(s->m);
    if (s->done.empty() && wait_us)
        s->cv_done.wait_for(lk, std::chrono::microseconds(wait_us), [&] { return !s->done.empty(); });
    uint32_t k = 0;
    while (k < max && !s->done.empty()) {
        Request *r = s->done.front();
        s->done.pop_front();
        sieve_result &o = out[k++];
        o.id = r->id;
        o.lo = r->lo;
        o.hi = r->hi;
        o.pi = r->pi;
        o.words = r->host;
        o.n_words = r->host ? r->n_words : 0;
        o.t_submit_ns = r->t_submit;
        o.t_admit_ns = r->t_admit;
        o.t_launch_ns = r->t_launch;
        o.t_done_ns = r->t_done;
        o.status = r->status;
        o.flags = r->flags;
        if (r->host)
            s->held[r->id] = r;
        else
            delete r;
    }
    *n_out = k;
    return SIEVE_OK;
}

int sieve_server_release(sieve_server *s, uint64_t id)
{
    if (!s)
        return SIEVE_EINVAL;
    std::lock_guard<std::mutex> g(s->m);
    auto it = s->held.find(id);
    if (it == s->held.end())
        return SIEVE_EINVAL;
    Request *r = it->second;
    s->arena.free(r->host_off, r->host_order);
    s->held.erase(it);
    delete r;
    s->cv_work.notify_one();  // freed host memory may let a request in
    return SIEVE_OK;
}

int sieve_server_get_stats(sieve_server *s, sieve_server_stats *out)
{
    if (!s || !out)
        return SIEVE_EINVAL;
    std::lock_guard<std::mutex> g(s->m);
    *out = s->stats;
    out->graph_captures = total_captures(s) - s->captures_at_create;
    return s->fatal;
}

int sieve_server_destroy(sieve_server *s)
{
    if (!s)
        return SIEVE_OK;
    {
        std::lock_guard<std::mutex> g(s->m);
        s->stop = true;
    }
    s->cv_work.notify_all();
    if (s->worker.joinable())
        s->worker.join();
    for (Lane &lane : s->lanes) {
        if (s->ctx)
            sv::engine_free(lane.eng);
        if (lane.h_pub)
            (void)hipHostFree(const_cast<unsigned long long *>(lane.h_pub));
        if (lane.copied)
            (void)hipEventDestroy(lane.copied);
        if (lane.stream)
            (void)hipStreamDestroy(lane.stream);
    }
    for (Request *r : s->done)
        delete r;
    for (auto &kv : s->held)
        delete kv.second;
    for (Request *r : s->pending)
        delete r;
    for (Request *r : s->admitted)
        delete r;
    if (s->d_pool)
        (void)hipFree(s->d_pool);
    if (s->h_arena)
        (void)hipHostFree(s->h_arena);
    if (s->ctx)
        sieve_destroy(s->ctx);
    delete s;
    return SIEVE_OK;
}

int sieve_serve_trace(int hip_device, const sieve_server_config *cfg, const uint64_t *lo, const uint64_t *hi,
                      const uint32_t *flags, const double *t_arrival_s, uint64_t n, uint64_t *pi_out,
                      double *latency_ms_out, sieve_server_stats *stats_out)
{
    if (!lo || !hi || !flags || !t_arrival_s || !pi_out || !latency_ms_out)
        return SIEVE_EINVAL;
    for (uint64_t i = 0; i < n; ++i) {
        if (lo[i] > hi[i])
            return SIEVE_EINVAL;
        if (hi[i] > SIEVE_MAX_HI)
            return SIEVE_ERANGE;
    }
    sieve_server *s = nullptr;
    if (int st = sieve_server_create(hip_device, cfg, &s))
        return st;
    std::atomic<int> sub_status{SIEVE_OK};
    // Request i is due at t0 + t_arrival_s[i]; its latency is measured from
    // then, so a submitter that falls behind shows up as queueing delay.
    const auto t0 = std::chrono::steady_clock::now();
    const uint64_t t0_ns = static_cast<uint64_t>(
        std::chrono::duration_cast<std::chrono::nanoseconds>(t0.time_since_epoch()).count());
    std::thread submitter([&] {
        for (uint64_t i = 0; i < n; ++i) {
            const auto due = t0 + std::chrono::nanoseconds(static_cast<int64_t>(t_arrival_s[i] * 1e9));
            // sleep most of the way, then spin for the last stretch
            const auto early = due - std::chrono::microseconds(200);
            if (std::chrono::steady_clock::now() < early)
                std::this_thread::sleep_until(early);
            while (std::chrono::steady_clock::now() < due) {
            }
            uint64_t id = 0;  // ids are 1, 2, ... in submission order
            const int st = sieve_server_submit(s, lo[i], hi[i], flags[i], &id);
            if (st != SIEVE_OK) {
                sub_status.store(st);
                return;
            }
        }
    });
    uint64_t got = 0;
    int status = SIEVE_OK;
    std::vector<sieve_result> buf(256);
    while (got < n) {
        uint32_t k = 0;
        sieve_server_poll(s, buf.data(), static_cast<uint32_t>(buf.size()), &k, 1000);
        for (uint32_t j = 0; j < k; ++j) {
            const sieve_result &r = buf[j];
            const uint64_t i = r.id - 1;
            if (r.status != SIEVE_OK)
                status = r.status;
            if (i < n) {
                pi_out[i] = r.pi;
                const double due_ns = static_cast<double>(t0_ns) + t_arrival_s[i] * 1e9;
                latency_ms_out[i] = (static_cast<double>(r.t_done_ns) - due_ns) * 1e-6;
            }
            if (r.words)
                sieve_server_release(s, r.id);
        }
        got += k;
        if (sub_status.load() != SIEVE_OK)
            break;
    }
    submitter.join();
    if (stats_out)
        sieve_server_get_stats(s, stats_out);
    sieve_server_destroy(s);
    const int sub = sub_status.load();
    return sub != SIEVE_OK ? sub : status;
}

}  // extern "C"
