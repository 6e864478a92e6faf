// Host runtime and C ABI of the exact range sieve (declared in sieve.h).
//
// The host side only validates arguments, plans segments and launches
// kernels: base primes, marking, counting and compaction all run on the
// device.  A context keeps the base-prime table resident in HBM (with a host
// mirror used for planning) so that repeated calls pay for it once.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "sieve_runtime.h"

namespace sv {

#define HIP_TRY SV_HIP_TRY

uint64_t isqrt_u64(uint64_t n)
{
    if (n < 2)
        return n;
    uint64_t r = static_cast<uint64_t>(std::sqrt(static_cast<double>(n)));
    while (r * r > n)
        --r;
    while ((r + 1) * (r + 1) <= n)
        ++r;
    return r;
}

// Largest segment (words) a workgroup with lds_bytes of LDS can hold.
uint32_t max_seg_words(uint32_t lds_bytes)
{
    uint32_t best = 0;
    for (uint32_t w = kSegGranuleWords; w <= sv::max_seg_words(); w += kSegGranuleWords)
        if (sv::lds_bytes_for(w) <= lds_bytes)
            best = w;
    return best;
}

int validate_tuning(const sieve_tuning &t, uint32_t lds_bytes)
{
    if (t.seg_bits) {
        if (t.seg_bits % (kSegGranuleWords * 32) != 0)
            return SIEVE_EINVAL;
        if (t.seg_bits / 32 > max_seg_words(lds_bytes))
            return SIEVE_EINVAL;
    }
    if (t.dense_limit > (1u << 20))
        return SIEVE_EINVAL;
    if (t.block_threads && t.block_threads != 256 && t.block_threads != 512 &&
        t.block_threads != 1024)
        return SIEVE_EINVAL;
    if (t.bucket_depth > (1u << 24))
        return SIEVE_EINVAL;
    if (t.wg_per_cu > 16)
        return SIEVE_EINVAL;
    return SIEVE_OK;
}

// Workgroup size for a segment of sw words: more waves share a larger
// segment's marking work (measured best: 1024 threads for 2^19 bits, 512
// from 2^14 to 2^18, 256 below).  Above 2^18 bits only two workgroups fit
// per CU, so they take 1024 threads to keep 32 wavefronts.
uint32_t default_threads(uint32_t sw)
{
    return sw > 8192 ? 1024u : (sw >= 512 ? 512u : 256u);
}

// Primes below the dense limit are marked a wavefront per prime: seg_bits /
// 512 (a prime there has at least ~500 multiples in the segment), but at
// least 128, so that on small segments the smallest primes' long walks are
// spread over a wavefront instead of one lane.
uint32_t default_dense_limit(uint32_t seg_bits)
{
    return std::max(seg_bits / 512, 128u);
}

int make_plan(uint64_t lo, uint64_t hi, const sieve_tuning *tu, uint32_t n_cu, uint32_t lds_bytes,
              sieve_plan_info *out)
{
    if (!out || lo > hi)
        return SIEVE_EINVAL;
    if (hi > SIEVE_MAX_HI)
        return SIEVE_ERANGE;
    sieve_tuning t{};
    if (tu)
        t = *tu;
    if (int st = validate_tuning(t, lds_bytes))
        return st;
    if (n_cu == 0)
        n_cu = 1;
    sieve_plan_info p{};
    p.nbits = hi / 2 - lo / 2;
    p.n_words = (p.nbits + 31) / 32;
    p.sqrt_bound = hi >= 2 ? isqrt_u64(hi - 1) : 0;
    const uint32_t cap = std::min(max_seg_words(lds_bytes), kDefaultMaxSegWords);
    if (cap == 0)
        return SIEVE_EINVAL;
    uint32_t sw;
    if (t.seg_bits) {
        sw = t.seg_bits / 32;
    } else {
        // enough segments for two workgroups per CU, within the LDS cap; a
        // power of two, so that hit buckets can split offsets with shifts
        const uint64_t want = (p.n_words + 2ull * n_cu - 1) / (2ull * n_cu);
        uint64_t pw = kSegGranuleWords;
        while (pw < want && pw < cap)
            pw *= 2;
        sw = static_cast<uint32_t>(std::min<uint64_t>(pw, cap));
    }
    if (!t.seg_bits && sw == kDefaultMaxSegWords && max_seg_words(lds_bytes) >= kWideSegWords) {
        // Long ranges take the widest segment (same occupancy, less set-up
        // per integer; measured 0.74 -> 0.70 ms on [2, 1e10), and with hit
        // buckets 2.72 -> 2.45 ms for 10^10 integers at 10^13, 14.7 -> 13.0
        // ms at 10^15).  Shorter ranges keep 2^19 bits: with under four
        // rounds of two workgroups per CU a wider segment mostly lengthens
        // the last round.
        const uint64_t sb = static_cast<uint64_t>(sw) * 32;
        const bool buckets = t.bucket_limit != 0xffffffffu &&
                             (t.bucket_limit ? true : p.sqrt_bound >= 2 * sb && p.nbits >= (1ull << 30));
        const uint64_t n_pow2 = (p.n_words + sw - 1) / sw;
        const uint64_t slots = 2ull * n_cu;  // two 1024-thread workgroups per CU
        if (n_pow2 >= 4 * slots) {
            sw = kWideSegWords;
        } else if (!buckets && n_pow2 > slots) {
            // two to four rounds: the same number of rounds, all of them
            // full, from the smallest segment that still fits them.  Just
            // past a full round (513 segments of 2^19 bits) the last round
            // would hold one segment; at [2, 1e9) (954 -> 1018 segments) the
            // gain is within noise.
            const uint64_t rounds = (n_pow2 + slots - 1) / slots;
            uint64_t bal = (p.n_words + rounds * slots - 1) / (rounds * slots);
            bal = (bal + kSegGranuleWords - 1) / kSegGranuleWords * kSegGranuleWords;
            if (bal < sw)
                sw = static_cast<uint32_t>(bal);
        }
    }
    p.seg_bits = sw * 32;
    p.dense_limit = t.dense_limit ? t.dense_limit : default_dense_limit(p.seg_bits);
    p.dense_limit = std::max(p.dense_limit, sv::kFirstMarkedPrime);
    p.block_threads = t.block_threads ? t.block_threads : default_threads(sw);
    p.n_segments = (p.n_words + sw - 1) / sw;
    // Hit buckets only pay when the largest base primes skip most segments:
    // from sqrt(hi) of two segments on (hi of about 1.55e12 with the widest
    // segment).  Measured for 10^10 integers on the widest segment, buckets
    // against none: 1.80 against 1.88 ms at 1.6e12 (sqrt(hi) 2.03
    // segments), 1.93 against 2.02 ms at 2e12, 2.46 against 3.72 ms at
    // 10^13; below two segments the gain comes and goes (1.64 against 1.62
    // ms at 10^12, 1.65 against 1.72 ms at 1.2e12).  The range must also be
    // long enough to amortise the fill launch and the overflow check's host
    // round trip (at least 2^30 odd integers).
    p.bucket_limit = 0;
    if (t.bucket_limit != 0xffffffffu && p.n_segments >= 2) {
        const uint64_t lim = std::max<uint64_t>(t.bucket_limit ? t.bucket_limit : p.seg_bits, p.seg_bits);
        const bool want = t.bucket_limit ? true : p.sqrt_bound >= 2ull * p.seg_bits && p.nbits >= (1ull << 30);
        if (want && lim <= p.sqrt_bound && lim < 0xffffffffull)
            p.bucket_limit = static_cast<uint32_t>(lim);
    }
    *out = p;
    return SIEVE_OK;
}

// The next per-call counter slot, once its previous user has finished.  A
// slot is all zero between calls (each call's last launch leaves it so); a
// call that failed before its launches were all enqueued left it dirty, and
// it is cleared on s first.  The caller marks the slot dirty until its last
// launch is enqueued.
int take_slot(sieve_ctx *c, hipStream_t s, uint32_t **words)
{
    // The first slot in turn that is free; only when every slot still has a
    // launch in flight (launches on several streams, one of them long) does
    // the call wait, for the oldest.
    int i = c->next_slot;
    for (int k = 0; k < sieve_ctx::kSlots; ++k) {
        const int j = (c->next_slot + k) % sieve_ctx::kSlots;
        if (!c->slot_used[j] || hipEventQuery(c->slot_done[j]) != hipErrorNotReady) {
            i = j;
            break;
        }
    }
    c->next_slot = (i + 1) % sieve_ctx::kSlots;
    if (c->slot_used[i])
        HIP_TRY(c, hipEventSynchronize(c->slot_done[i]));
    c->slot_used[i] = false;
    *words = c->d_ctr + static_cast<size_t>(i) * kCounterWords;
    if (c->slot_dirty[i])
        HIP_TRY(c, hipMemsetAsync(*words, 0, kCounterWords * sizeof(uint32_t), s));
    c->slot_dirty[i] = true;
    return i;
}

// The pinned word the last launch of a call publishes its count to: reset
// to a value no count can take before the launch, read after the stream
// synchronises.
constexpr uint64_t kUnpublished = ~0ull;

volatile uint64_t *published(sieve_ctx *c)
{
    return reinterpret_cast<volatile uint64_t *>(c->h_ctr);
}

// Workgroups that fit on the device at once for a plan.
uint32_t resident_blocks(const sieve_ctx *c, const sieve_plan_info &pl, bool write)
{
    uint32_t per_cu = sv::range_blocks_per_cu(pl.seg_bits / 32, pl.block_threads, write);
    if (c->tuning.wg_per_cu)
        per_cu = std::min(per_cu, c->tuning.wg_per_cu);
    return std::max(per_cu, 1u) * c->n_cu;
}

// Build the device table of all odd primes <= limit (limit >= 2^16 - 1).
int build_primes(sieve_ctx *c, uint64_t limit)
{
    hipStream_t s = c->stream;
    uint32_t *d_boot = nullptr, *d_small = nullptr;
    double *d_boot_inv = nullptr;
    HIP_TRY(c, hipMalloc(&d_boot, sv::kBootstrapOddPrimes * sizeof(uint32_t)));
    HIP_TRY(c, hipMalloc(&d_small, 4 * sizeof(uint32_t)));
    HIP_TRY(c, hipMalloc(&d_boot_inv, sv::kBootstrapOddPrimes * sizeof(double)));
    int st = SIEVE_OK;
    uint32_t *d_words = nullptr, *d_tmp = nullptr, *d_out = nullptr;
    double *d_out_inv = nullptr;
    uint32_t total = 0;
    do {
        hipError_t e = sv::launch_bootstrap_primes(d_boot, d_small, s);
        if (e == hipSuccess)
            e = sv::launch_reciprocals(d_boot, sv::kBootstrapOddPrimes, d_boot_inv, s);
        uint32_t boot_n = 0;
        if (e == hipSuccess)
            e = hipMemcpyAsync(&boot_n, d_small, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_EDEVICE;
            break;
        }
        if (boot_n != sv::kBootstrapOddPrimes) {
            st = SIEVE_EDEVICE;
            break;
        }
        // The range sieve of [0, limit + 1) with the bootstrap primes as base
        // primes, then a compaction of its bitmap.
        const uint64_t hi = limit + 1;
        sieve_plan_info pl{};
        st = make_plan(0, hi, nullptr, c->n_cu, c->lds_max, &pl);
        if (st)
            break;
        const uint64_t r = pl.sqrt_bound;  // < 2^16 since limit < 2^32
        std::vector<uint32_t> boot(sv::kBootstrapOddPrimes);
        e = hipMemcpy(boot.data(), d_boot, boot.size() * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_EDEVICE;
            break;
        }
        const uint32_t n_odd = static_cast<uint32_t>(std::upper_bound(boot.begin(), boot.end(), r) - boot.begin());
        const uint32_t n_mark = n_odd > sv::kPresievePrimes ? n_odd - sv::kPresievePrimes : 0;
        const uint32_t n_dense_all = static_cast<uint32_t>(
            std::lower_bound(boot.begin(), boot.end(), pl.dense_limit) - boot.begin());
        const uint32_t n_dense = std::min(n_mark, n_dense_all > sv::kPresievePrimes ? n_dense_all - sv::kPresievePrimes : 0u);
        const uint64_t out_cap = static_cast<uint64_t>(1.3 * hi / std::log(static_cast<double>(hi))) + 1024;
        if ((e = hipMalloc(&d_words, pl.n_words * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&d_tmp, sv::compact_tmp_words(pl.n_words) * sizeof(uint32_t))) != hipSuccess ||
            (e = hipMalloc(&d_out, out_cap * sizeof(uint32_t))) != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_ENOMEM;
            break;
        }
        uint32_t *slot = nullptr;
        const int si = take_slot(c, s, &slot);
        if (si < 0) {
            st = si;
            break;
        }
        sv::RangeArgs ra{1, pl.nbits, pl.n_words, d_words, slot, false, true, nullptr, nullptr, nullptr, 0};
        sv::PrimeArgs pa{d_boot + sv::kPresievePrimes, d_boot_inv + sv::kPresievePrimes, n_dense, n_mark};
        e = sv::launch_range(ra, pa, pl.seg_bits / 32, pl.block_threads,
                             static_cast<uint32_t>(pl.n_segments), resident_blocks(c, pl, true), s);
        if (e == hipSuccess)
            c->slot_dirty[si] = false;
        if (e == hipSuccess)
            e = hipEventRecord(c->slot_done[si], s);
        c->slot_used[si] = true;
        if (e == hipSuccess)
            e = sv::launch_compact(d_words, pl.n_words, 1, d_tmp, d_out, d_small, s);
        if (e == hipSuccess)
            e = hipMemcpyAsync(&total, d_small, sizeof(uint32_t), hipMemcpyDeviceToHost, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_EDEVICE;
            break;
        }
        if (total > out_cap) {
            st = SIEVE_EDEVICE;
            break;
        }
        std::vector<uint32_t> h(total);
        e = hipMemcpy(h.data(), d_out, total * sizeof(uint32_t), hipMemcpyDeviceToHost);
        if (e == hipSuccess)
            e = hipMalloc(&d_out_inv, std::max<uint32_t>(total, 1) * sizeof(double));
        if (e == hipSuccess)
            e = sv::launch_reciprocals(d_out, total, d_out_inv, s);
        if (e == hipSuccess)
            e = hipStreamSynchronize(s);
        if (e != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_EDEVICE;
            break;
        }
        // the bitmap of [0, limit] has no bit for 2: the list is the odd primes.
        // Launches on other streams may still read the old table.
        e = hipDeviceSynchronize();
        if (e != hipSuccess) {
            c->last_hip = e;
            st = SIEVE_EDEVICE;
            break;
        }
        if (c->d_primes)
            (void)hipFree(c->d_primes);
        if (c->d_inv)
            (void)hipFree(c->d_inv);
        c->d_primes = d_out;
        c->d_inv = d_out_inv;
        d_out = nullptr;
        d_out_inv = nullptr;
        c->h_primes.swap(h);
        c->h_recip_prefix.assign(c->h_primes.size() + 1, 0.0);
        for (size_t i = 0; i < c->h_primes.size(); ++i)
            c->h_recip_prefix[i + 1] = c->h_recip_prefix[i] + 1.0 / c->h_primes[i];
        c->h_pi_index.assign((limit >> kPiIndexShift) + 2, 0);
        for (size_t k = 0, i = 0; k < c->h_pi_index.size(); ++k) {
            while (i < c->h_primes.size() && (c->h_primes[i] >> kPiIndexShift) < k)
                ++i;
            c->h_pi_index[k] = static_cast<uint32_t>(i);
        }
        c->primes_limit = limit;
    } while (false);
    (void)hipFree(d_boot);
    (void)hipFree(d_small);
    (void)hipFree(d_boot_inv);
    if (d_out_inv)
        (void)hipFree(d_out_inv);
    if (d_words)
        (void)hipFree(d_words);
    if (d_tmp)
        (void)hipFree(d_tmp);
    if (d_out)
        (void)hipFree(d_out);
    return st;
}

int ensure_primes(sieve_ctx *c, uint64_t bound)
{
    if (bound <= c->primes_limit)
        return SIEVE_OK;
    if (bound > kMaxPrimeLimit)
        return SIEVE_ERANGE;
    uint64_t lim = std::max<uint64_t>(bound, 2 * c->primes_limit);
    lim = std::max<uint64_t>(lim, sv::kBootstrapLimit);
    lim = std::min<uint64_t>(lim, kMaxPrimeLimit);
    return build_primes(c, lim);
}

// Marking primes for sieving with base-prime bound r: (count, dense count).
// Number of odd primes <= r in the context's table (r <= primes_limit): the
// coarse index narrows the search to the primes of one 2^8-wide block.
uint32_t odd_primes_upto(const sieve_ctx *c, uint64_t r)
{
    const auto &v = c->h_primes;
    const uint64_t k = r >> kPiIndexShift;
    if (k + 1 >= c->h_pi_index.size())
        return static_cast<uint32_t>(std::upper_bound(v.begin(), v.end(), r) - v.begin());
    const auto first = v.begin() + c->h_pi_index[k], last = v.begin() + c->h_pi_index[k + 1];
    return static_cast<uint32_t>(std::upper_bound(first, last, r) - v.begin());
}

void marking_primes(const sieve_ctx *c, uint64_t r, uint32_t dense_limit, uint32_t *n_mark,
                    uint32_t *n_dense)
{
    const uint32_t n_odd = odd_primes_upto(c, r);
    *n_mark = n_odd > sv::kPresievePrimes ? n_odd - sv::kPresievePrimes : 0;
    const uint32_t nd = odd_primes_upto(c, dense_limit - 1);
    *n_dense = std::min(*n_mark, nd > sv::kPresievePrimes ? nd - sv::kPresievePrimes : 0u);
}

namespace {

// The plain path with large-prime hit buckets: the range is cut into
// windows of W segments (the bucket pool holds W buckets); per window, the
// fill kernel sorts the large primes' hits into buckets, then the range
// kernel sieves the window's segments with the small and medium primes plus
// its buckets.  Counts accumulate in the call's slot.  An overflowing bucket
// is detected after the last window and the call is redone with twice the
// depth.
int run_range_bucketed(sieve_ctx *c, const sieve_plan_info &pl, uint64_t lo, uint32_t *d_words,
                       uint64_t *pi_out, hipStream_t s, uint32_t n_mark, uint32_t n_dense)
{
    const auto &v = c->h_primes;
    const uint32_t sw = pl.seg_bits / 32;
    // marking primes [0, n_small) are scanned per segment; [n_small, n_mark) are bucketed
    const uint32_t n_below = static_cast<uint32_t>(std::lower_bound(v.begin(), v.end(), pl.bucket_limit) - v.begin());
    const uint32_t n_small = std::min(n_mark, n_below > kPresievePrimes ? n_below - kPresievePrimes : 0u);
    const uint32_t n_large = n_mark - n_small;
    // expected hits per segment: (8/15) * (seg_bits / p) summed over the large primes
    const double recip = c->h_recip_prefix[kPresievePrimes + n_mark] - c->h_recip_prefix[kPresievePrimes + n_small];
    const double expect = (8.0 / 15.0) * pl.seg_bits * recip;
    uint64_t depth = c->tuning.bucket_depth
                         ? c->tuning.bucket_depth
                         : static_cast<uint64_t>(expect + 6.0 * std::sqrt(expect) + 64.0);
    depth = (depth + 63) / 64 * 64;
    const uint64_t first_odd = (lo & ~1ull) + 1;
    for (;;) {
        const uint64_t win = std::max<uint64_t>(1, std::min<uint64_t>(pl.n_segments, kBucketPoolBytes / (4 * depth)));
        if (int st = grow(c, c->b_buckets, win * depth * sizeof(uint32_t)))
            return st;
        if (int st = grow(c, c->b_bcount, (win + 1) * sizeof(uint32_t)))
            return st;
        uint32_t *buckets = static_cast<uint32_t *>(c->b_buckets.p);
        uint32_t *bcount = static_cast<uint32_t *>(c->b_bcount.p);
        uint32_t *overflow = bcount + win;
        uint32_t *slot = nullptr;
        const int si = take_slot(c, s, &slot);
        if (si < 0)
            return si;
        HIP_TRY(c, hipMemsetAsync(overflow, 0, sizeof(uint32_t), s));
        *published(c) = kUnpublished;
        c->ev_valid = false;
        if (c->timing)
            HIP_TRY(c, hipEventRecord(c->ev_start, s));
        for (uint64_t w0 = 0; w0 < pl.n_segments; w0 += win) {
            const uint32_t segs = static_cast<uint32_t>(std::min<uint64_t>(win, pl.n_segments - w0));
            const uint64_t word0 = w0 * sw;
            const uint64_t bits_w = std::min<uint64_t>(static_cast<uint64_t>(segs) * pl.seg_bits, pl.nbits - word0 * 32);
            const uint64_t fo = first_odd + 64 * word0;
            HIP_TRY(c, hipMemsetAsync(bcount, 0, segs * sizeof(uint32_t), s));
            HIP_TRY(c, sv::launch_bucket_fill(c->d_primes + kPresievePrimes + n_small,
                                              c->d_inv + kPresievePrimes + n_small, n_large, fo, pl.seg_bits, segs,
                                              buckets, bcount, static_cast<uint32_t>(depth), overflow, s));
            const bool last = w0 + win >= pl.n_segments;
            sv::RangeArgs ra{fo, bits_w, (bits_w + 31) / 32, d_words ? d_words + word0 : nullptr,
                             slot, pi_out != nullptr, last, pi_out && last ? c->d_pub : nullptr,
                             buckets, bcount, static_cast<uint32_t>(depth)};
            sv::PrimeArgs pa{c->d_primes + kPresievePrimes, c->d_inv + kPresievePrimes, std::min(n_dense, n_small),
                             n_small};
            sieve_plan_info wp = pl;
            wp.n_segments = segs;
            HIP_TRY(c, sv::launch_range(ra, pa, sw, pl.block_threads, segs,
                                        resident_blocks(c, wp, d_words != nullptr), s));
        }
        c->slot_dirty[si] = false;
        if (c->timing) {
            HIP_TRY(c, hipEventRecord(c->ev_stop, s));
            c->ev_valid = true;
        }
        uint32_t *h_flag = c->h_ctr + 16;
        HIP_TRY(c, hipMemcpyAsync(h_flag, overflow, sizeof(uint32_t), hipMemcpyDeviceToHost, s));
        HIP_TRY(c, hipEventRecord(c->slot_done[si], s));
        c->slot_used[si] = true;
        HIP_TRY(c, hipStreamSynchronize(s));
        if (*h_flag == 0) {
            if (pi_out) {
                const uint64_t v = *published(c);
                if (v == kUnpublished)
                    return SIEVE_EDEVICE;
                *pi_out = v;  // odd primes only
            }
            return SIEVE_OK;
        }
        if (depth >= (1ull << 26))
            return SIEVE_EOVERFLOW;
        depth *= 2;
    }
}

}  // namespace

namespace {

// One plain launch of a planned range without buckets on s: the count of odd
// primes is published to *d_pub (a device-visible pinned word) when d_pub is
// not null.  timed: bracket the launch with the context's timing events.
int enqueue_plain(sieve_ctx *c, const sieve_plan_info &pl, uint64_t lo, uint32_t *d_words,
                  unsigned long long *d_pub, hipStream_t s, bool timed, uint32_t n_mark, uint32_t n_dense,
                  int *slot_out = nullptr)
{
    uint32_t *slot = nullptr;
    const int si = take_slot(c, s, &slot);
    if (si < 0)
        return si;
    if (slot_out)
        *slot_out = si;
    sv::RangeArgs ra{(lo & ~1ull) + 1, pl.nbits, pl.n_words, d_words, slot, d_pub != nullptr, true,
                     d_pub, nullptr, nullptr, 0};
    sv::PrimeArgs pa{c->d_primes + sv::kPresievePrimes, c->d_inv + sv::kPresievePrimes, n_dense, n_mark};
    if (timed) {
        c->ev_valid = false;
        HIP_TRY(c, hipEventRecord(c->ev_start, s));
    }
    HIP_TRY(c, sv::launch_range(ra, pa, pl.seg_bits / 32, pl.block_threads,
                                static_cast<uint32_t>(pl.n_segments),
                                resident_blocks(c, pl, d_words != nullptr), s));
    c->slot_dirty[si] = false;
    if (timed) {
        HIP_TRY(c, hipEventRecord(c->ev_stop, s));
        c->ev_valid = true;
    }
    HIP_TRY(c, hipEventRecord(c->slot_done[si], s));
    c->slot_used[si] = true;
    return SIEVE_OK;
}

// The count a plain launch in counter slot si publishes: spin on the pinned
// word, which the launch's last workgroup writes as it leaves, instead of
// synchronising the stream (the wake-up costs several microseconds).  Every
// few hundred reads the slot's completion event is queried, so a launch that
// ends without publishing (a failed launch) is reported instead of waited on
// forever; the stream is then synchronised to collect its error.
int wait_published(sieve_ctx *c, int si, hipStream_t s, uint64_t *v)
{
    for (uint32_t k = 1;; ++k) {
        const uint64_t x = *published(c);
        if (x != kUnpublished) {
            *v = x;
            return SIEVE_OK;
        }
        if ((k & 255) == 0 && hipEventQuery(c->slot_done[si]) != hipErrorNotReady) {
            HIP_TRY(c, hipStreamSynchronize(s));
            const uint64_t y = *published(c);
            if (y == kUnpublished)
                return SIEVE_EDEVICE;
            *v = y;
            return SIEVE_OK;
        }
        __builtin_ia32_pause();
    }
}

}  // namespace

int run_range(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, uint64_t *pi_out,
              hipStream_t s)
{
    sieve_plan_info pl{};
    if (int st = make_plan(lo, hi, &c->tuning, c->n_cu, c->lds_max, &pl))
        return st;
    const uint64_t two = (lo <= 2 && 2 < hi) ? 1 : 0;
    if (pl.nbits == 0) {
        if (pi_out)
            *pi_out = two;
        return SIEVE_OK;
    }
    if (pl.n_segments > 0xffffffffull)
        return SIEVE_ERANGE;
    HIP_TRY(c, hipSetDevice(c->device));
    if (int st = ensure_primes(c, pl.sqrt_bound))
        return st;
    uint32_t n_mark = 0, n_dense = 0;
    marking_primes(c, pl.sqrt_bound, pl.dense_limit, &n_mark, &n_dense);
    if (pl.bucket_limit) {
        uint64_t pi = 0;
        if (int st = run_range_bucketed(c, pl, lo, d_words, pi_out ? &pi : nullptr, s, n_mark, n_dense))
            return st;
        if (pi_out)
            *pi_out = pi + two;
        return SIEVE_OK;
    }
    if (pi_out)
        *published(c) = kUnpublished;
    int si = -1;
    if (int st = enqueue_plain(c, pl, lo, d_words, pi_out ? c->d_pub : nullptr, s, c->timing, n_mark, n_dense,
                               &si))
        return st;
    if (pi_out) {
        // the count is known once published; a bitmap's words follow in
        // stream order like any launch on s
        uint64_t v = kUnpublished;
        if (int st = wait_published(c, si, s, &v))
            return st;
        *pi_out = v + two;
    }
    return SIEVE_OK;
}

bool range_async_ok(const sieve_ctx *c, uint64_t lo, uint64_t hi)
{
    sieve_plan_info pl{};
    return make_plan(lo, hi, &c->tuning, c->n_cu, c->lds_max, &pl) == SIEVE_OK && pl.nbits != 0 &&
           !pl.bucket_limit && pl.n_segments <= 0xffffffffull;
}

int range_async(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, unsigned long long *d_pub,
                hipStream_t s)
{
    sieve_plan_info pl{};
    if (int st = make_plan(lo, hi, &c->tuning, c->n_cu, c->lds_max, &pl))
        return st;
    if (pl.nbits == 0 || pl.bucket_limit || pl.n_segments > 0xffffffffull)
        return kNotAsync;
    HIP_TRY(c, hipSetDevice(c->device));
    if (int st = ensure_primes(c, pl.sqrt_bound))
        return st;
    uint32_t n_mark = 0, n_dense = 0;
    marking_primes(c, pl.sqrt_bound, pl.dense_limit, &n_mark, &n_dense);
    return enqueue_plain(c, pl, lo, d_words, d_pub, s, false, n_mark, n_dense);
}

int grow(sieve_ctx *c, DevBuf &b, size_t bytes)
{
    if (b.bytes >= bytes)
        return SIEVE_OK;
    const size_t want = std::max(bytes, b.bytes * 2);
    if (b.p)
        HIP_TRY(c, hipFree(b.p));
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipMalloc(&b.p, want);
    if (e != hipSuccess) {
        c->last_hip = e;
        b.p = nullptr;
        return SIEVE_ENOMEM;
    }
    b.bytes = want;
    return SIEVE_OK;
}

int grow_host(sieve_ctx *c, HostBuf &b, size_t bytes)
{
    if (b.bytes >= bytes)
        return SIEVE_OK;
    const size_t want = std::max(bytes, b.bytes * 2);
    if (b.p)
        HIP_TRY(c, hipHostFree(b.p));
    b.p = nullptr;
    b.d = nullptr;
    b.bytes = 0;
    hipError_t e = hipHostMalloc(&b.p, want, hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess)
        e = hipHostGetDevicePointer(&b.d, b.p, 0);
    if (e != hipSuccess) {
        c->last_hip = e;
        if (b.p)
            (void)hipHostFree(b.p);
        b.p = nullptr;
        b.d = nullptr;
        return e == hipErrorOutOfMemory ? SIEVE_ENOMEM : SIEVE_EDEVICE;
    }
    b.bytes = want;
    return SIEVE_OK;
}

namespace {

void drop_graph(BatchEngine &e, int v)
{
    if (e.exec[v])
        (void)hipGraphExecDestroy(e.exec[v]);
    if (e.graph[v])
        (void)hipGraphDestroy(e.graph[v]);
    e.exec[v] = nullptr;
    e.graph[v] = nullptr;
}

// Capture the batch launch sequence on the context's own stream (capture runs
// nothing) and instantiate it into the engine's slot for k.small; the graph
// may then be launched on any stream.
int capture_batch_graph(sieve_ctx *c, BatchEngine &eng, const GraphKey &k)
{
    const int v = k.small ? 1 : 0;
    drop_graph(eng, v);
    hipStream_t cs = c->stream;
    HIP_TRY(c, hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
    hipError_t e = sv::launch_batch(k.h_blob, static_cast<sv::BatchHeader *>(const_cast<void *>(k.blob)),
                                    k.max_intervals, static_cast<const uint32_t *>(k.primes),
                                    static_cast<const double *>(k.inv), k.words,
                                    static_cast<uint32_t *>(const_cast<void *>(k.item_counts)),
                                    static_cast<unsigned long long *>(const_cast<void *>(k.counts)),
                                    k.seg_words, k.threads, k.blocks, k.small, cs);
    hipGraph_t g = nullptr;
    hipError_t e2 = hipStreamEndCapture(cs, &g);
    if (e == hipSuccess)
        e = e2;
    if (e == hipSuccess)
        e = hipGraphInstantiate(&eng.exec[v], g, nullptr, nullptr, 0);
    if (e != hipSuccess) {
        if (g)
            (void)hipGraphDestroy(g);
        eng.exec[v] = nullptr;
        c->last_hip = e;
        return SIEVE_EDEVICE;
    }
    eng.graph[v] = g;
    eng.key[v] = k;
    ++eng.captures;
    return SIEVE_OK;
}

}  // namespace

int engine_init(sieve_ctx *c, BatchEngine &e)
{
    HIP_TRY(c, hipEventCreateWithFlags(&e.done, hipEventDisableTiming));
    return SIEVE_OK;
}

namespace {
// Byte layout of a staged blob for n intervals and `items` work items.
uint64_t blob_items_offset(uint32_t n)
{
    const uint64_t iv_bytes = static_cast<uint64_t>(n) * sizeof(sv::BatchInterval);
    return kBlobIntervalOff + (iv_bytes + kBlobAlign - 1) / kBlobAlign * kBlobAlign;
}
uint64_t blob_bytes(uint32_t n, uint64_t items)  // whole 16-byte chunks, as the stage kernel copies
{
    return (blob_items_offset(n) + std::max<uint64_t>(1, items) * sizeof(uint32_t) + 15) / 16 * 16;
}
}  // namespace

int engine_reserve(sieve_ctx *c, BatchEngine &e, uint32_t n, uint64_t items)
{
    const uint64_t bytes = blob_bytes(n, items);
    if (int st = grow_host(c, e.s_blob, bytes))
        return st;
    if (int st = grow(c, e.blob, bytes))
        return st;
    if (int st = grow(c, e.item_counts, std::max<uint64_t>(1, items) * sizeof(uint32_t)))
        return st;
    return grow_host(c, e.s_counts, std::max<uint64_t>(1, n) * sizeof(unsigned long long));
}

void engine_free(BatchEngine &e)
{
    if (e.done && e.pending)
        (void)hipEventSynchronize(e.done);
    drop_graph(e, 0);
    drop_graph(e, 1);
    for (DevBuf *b : {&e.blob, &e.item_counts})
        if (b->p)
            (void)hipFree(b->p);
    for (HostBuf *b : {&e.s_blob, &e.s_counts})
        if (b->p)
            (void)hipHostFree(b->p);
    if (e.done)
        (void)hipEventDestroy(e.done);
    e = BatchEngine();
}

uint32_t batch_seg_words(const sieve_ctx *c)
{
    // a batch never uses hit buckets, so it takes the widest segment two
    // workgroups per CU can hold (measured 3.52 -> 3.3 ms on 4096 intervals)
    const uint32_t cap = std::min(max_seg_words(c->lds_max), kWideSegWords);
    return c->tuning.seg_bits ? c->tuning.seg_bits / 32 : cap;
}

uint64_t engine_device_bytes(uint32_t n, uint64_t items)
{
    return blob_bytes(n, items) + std::max<uint64_t>(1, items) * sizeof(uint32_t);
}

int engine_stage(sieve_ctx *c, BatchEngine &e, const sieve_interval *iv, uint32_t n, uint32_t *d_words,
                 uint64_t total_words)
{
    if (int st = validate_tuning(c->tuning, c->lds_max))
        return st;
    const uint32_t sw = batch_seg_words(c);
    const uint32_t dense_limit = std::max(c->tuning.dense_limit ? c->tuning.dense_limit : default_dense_limit(sw * 32),
                                          sv::kFirstMarkedPrime);
    const uint32_t threads = c->tuning.block_threads ? c->tuning.block_threads : default_threads(sw);
    std::vector<std::pair<uint64_t, uint64_t>> spans;
    uint64_t max_bound = 0, items = 0;
    e.bound.resize(n);
    for (uint32_t i = 0; i < n; ++i) {
        if (iv[i].lo > iv[i].hi)
            return SIEVE_EINVAL;
        if (iv[i].hi > SIEVE_MAX_HI)
            return SIEVE_ERANGE;
        const uint64_t nw = sieve_bitmap_words(iv[i].lo, iv[i].hi);
        if (iv[i].flags & SIEVE_WANT_BITMAP) {
            if (nw && !d_words)
                return SIEVE_EINVAL;
            if (iv[i].word_offset > total_words || nw > total_words - iv[i].word_offset)
                return SIEVE_EBUFSZ;
            if (nw)
                spans.emplace_back(iv[i].word_offset, iv[i].word_offset + nw);
        }
        e.bound[i] = iv[i].hi >= 2 ? isqrt_u64(iv[i].hi - 1) : 0;
        max_bound = std::max(max_bound, e.bound[i]);
        items += (nw + sw - 1) / sw;
    }
    std::sort(spans.begin(), spans.end());
    for (size_t i = 1; i < spans.size(); ++i)
        if (spans[i].first < spans[i - 1].second)
            return SIEVE_EINVAL;
    if (items > 0xffffffffull)
        return SIEVE_ERANGE;
    if (engine_device_bytes(n, items) > c->hbm_budget)
        return SIEVE_ENOMEM;

    HIP_TRY(c, hipSetDevice(c->device));
    if (int st = ensure_primes(c, max_bound))
        return st;
    // The staging buffers may still be read by the previous launch's stage kernel.
    if (e.pending)
        HIP_TRY(c, hipEventSynchronize(e.done));
    e.pending = false;
    const uint64_t bytes = blob_bytes(n, items);
    if (int st = grow_host(c, e.s_blob, bytes))
        return st;
    char *blob = static_cast<char *>(e.s_blob.p);

    // Intervals whose segments carry the most base primes go first, so the
    // cheapest work items are the ones left at the end of the queue.
    std::memset(blob, 0, kBlobIntervalOff);  // header and work queues
    sv::BatchInterval *h_iv = reinterpret_cast<sv::BatchInterval *>(blob + kBlobIntervalOff);
    uint32_t *h_item = reinterpret_cast<uint32_t *>(blob + blob_items_offset(n));
    // queue order: intervals by power-of-two class of their marking-prime
    // count, largest first, input order within a class (a two-pass
    // counting sort, linear in n)
    e.order.resize(n);
    e.nmark.resize(n);
    const uint32_t nd_all = odd_primes_upto(c, dense_limit - 1);
    const uint32_t n_dense_max = nd_all > sv::kPresievePrimes ? nd_all - sv::kPresievePrimes : 0u;
    uint32_t first_of[34] = {};
    for (uint32_t i = 0; i < n; ++i) {
        const uint32_t n_odd = odd_primes_upto(c, e.bound[i]);
        e.nmark[i] = n_odd > sv::kPresievePrimes ? n_odd - sv::kPresievePrimes : 0;
        ++first_of[32 - __builtin_clz(e.nmark[i] + 1)];
    }
    for (uint32_t k = 33, at = 0; k-- > 0;) {
        const uint32_t cnt = first_of[k];
        first_of[k] = at;
        at += cnt;
    }
    for (uint32_t i = 0; i < n; ++i)
        e.order[first_of[32 - __builtin_clz(e.nmark[i] + 1)]++] = i;
    uint32_t next = 0;
    for (uint32_t j = 0; j < n; ++j) {
        const uint32_t i = e.order[j];
        const uint64_t lo = iv[i].lo, hi = iv[i].hi;
        sv::BatchInterval b;
        b.first_odd = (lo & ~1ull) + 1;
        b.nbits = hi / 2 - lo / 2;
        b.n_words = (b.nbits + 31) / 32;
        b.word_offset = (iv[i].flags & SIEVE_WANT_BITMAP) ? iv[i].word_offset : ~0ull;
        b.n_primes = e.nmark[i];
        b.n_dense = std::min(e.nmark[i], n_dense_max);
        b.seg_begin = next;
        b.pad = 0;
        h_iv[i] = b;
        const uint32_t segs = static_cast<uint32_t>((b.n_words + sw - 1) / sw);
        std::fill(h_item + next, h_item + next + segs, i);
        next += segs;
    }
    sv::BatchHeader *h_hdr = reinterpret_cast<sv::BatchHeader *>(blob);
    h_hdr->n_intervals = n;
    h_hdr->n_items = static_cast<uint32_t>(items);
    h_hdr->seg_words = sw;
    h_hdr->blob_chunks = static_cast<uint32_t>(bytes / 16);
    h_hdr->iv_off = kBlobIntervalOff;
    h_hdr->item_off = blob_items_offset(n);
    e.blob_used = bytes;
    e.n = n;
    e.items = items;
    e.seg_words = sw;
    e.dense_limit = dense_limit;
    e.threads = threads;
    e.small = max_bound < (1ull << 24);
    return SIEVE_OK;
}

int engine_graph(sieve_ctx *c, BatchEngine &e, uint32_t *d_words, bool small)
{
    uint32_t per_cu = std::max(1u, sv::batch_blocks_per_cu(e.seg_words, e.threads));
    if (c->tuning.wg_per_cu)
        per_cu = std::min(per_cu, c->tuning.wg_per_cu);
    GraphKey k{};
    k.h_blob = e.s_blob.d;
    k.blob = e.blob.p;
    k.counts = e.s_counts.d;
    k.item_counts = e.item_counts.p;
    k.primes = c->d_primes + sv::kPresievePrimes;
    k.inv = c->d_inv + sv::kPresievePrimes;
    k.words = d_words;
    k.seg_words = e.seg_words;
    k.threads = e.threads;
    k.blocks = per_cu * c->n_cu;
    k.max_intervals = static_cast<uint32_t>(e.s_counts.bytes / sizeof(unsigned long long));
    k.small = small;
    const int v = small ? 1 : 0;
    if (!e.exec[v] || !(e.key[v] == k))
        return capture_batch_graph(c, e, k);
    return SIEVE_OK;
}

int engine_launch(sieve_ctx *c, BatchEngine &e, uint32_t *d_words, hipStream_t s, bool timed)
{
    const uint32_t n = e.n;
    if (int st = engine_reserve(c, e, n, e.items))
        return st;
    if (int st = engine_graph(c, e, d_words, e.small))
        return st;
    if (timed) {
        c->ev_valid = false;
        HIP_TRY(c, hipEventRecord(c->ev_start, s));
    }
    HIP_TRY(c, hipGraphLaunch(e.exec[e.small ? 1 : 0], s));
    if (timed) {
        HIP_TRY(c, hipEventRecord(c->ev_stop, s));
        c->ev_valid = true;
    }
    HIP_TRY(c, hipEventRecord(e.done, s));
    e.pending = true;
    return SIEVE_OK;
}

}  // namespace

extern "C" {

const char *sieve_strerror(int status)
{
    switch (status) {
    case SIEVE_OK: return "success";
    case SIEVE_EINVAL: return "invalid argument";
    case SIEVE_ERANGE: return "range outside [0, 10^15]";
    case SIEVE_ENOMEM: return "out of memory or over the HBM budget";
    case SIEVE_EBUFSZ: return "output buffer too small";
    case SIEVE_EDEVICE: return "HIP device error";
    case SIEVE_ENODEV: return "no gfx950 device";
    case SIEVE_EOVERFLOW: return "bucket pool overflow";
    default: return "unknown status";
    }
}

uint64_t sieve_bitmap_words(uint64_t lo, uint64_t hi)
{
    if (lo >= hi)
        return 0;
    return (hi / 2 - lo / 2 + 31) / 32;
}

int sieve_plan(uint64_t lo, uint64_t hi, const sieve_tuning *tuning, uint32_t n_cu, uint32_t lds_bytes,
               sieve_plan_info *out)
{
    return sv::make_plan(lo, hi, tuning, n_cu, lds_bytes, out);
}

int sieve_create(sieve_ctx **out, int hip_device, uint64_t hbm_budget_bytes)
{
    if (!out)
        return SIEVE_EINVAL;
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n <= 0 || hip_device < 0 || hip_device >= n)
        return SIEVE_ENODEV;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, hip_device) != hipSuccess)
        return SIEVE_ENODEV;
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return SIEVE_ENODEV;
    sieve_ctx *c = new (std::nothrow) sieve_ctx();
    if (!c)
        return SIEVE_ENOMEM;
    c->device = hip_device;
    c->n_cu = static_cast<uint32_t>(prop.multiProcessorCount);
    c->lds_max = static_cast<uint32_t>(prop.sharedMemPerBlock);
    c->lds_per_cu = static_cast<uint32_t>(prop.maxSharedMemoryPerMultiProcessor);
    if (c->lds_per_cu < c->lds_max)
        c->lds_per_cu = c->lds_max;
    if (hbm_budget_bytes)
        c->hbm_budget = hbm_budget_bytes;
    int st = SIEVE_OK;
    hipError_t e = hipSetDevice(hip_device);
    if (e == hipSuccess)
        e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
    if (e == hipSuccess)
        e = hipMalloc(&c->d_ctr, sieve_ctx::kSlots * sv::kCounterWords * sizeof(uint32_t));
    for (int i = 0; i < sieve_ctx::kSlots && e == hipSuccess; ++i)
        e = hipEventCreateWithFlags(&c->slot_done[i], hipEventDisableTiming);
    if (e == hipSuccess)
        e = hipHostMalloc(&c->h_ctr, 64 * sizeof(uint32_t), hipHostMallocMapped | hipHostMallocCoherent);
    if (e == hipSuccess)
        e = hipHostGetDevicePointer(reinterpret_cast<void **>(&c->d_pub), c->h_ctr, 0);
    if (e == hipSuccess)
        e = hipMemsetAsync(c->d_ctr, 0, sieve_ctx::kSlots * sv::kCounterWords * sizeof(uint32_t), c->stream);
    if (e == hipSuccess)
        e = hipStreamSynchronize(c->stream);
    if (e == hipSuccess)
        e = hipEventCreate(&c->ev_start);
    if (e == hipSuccess)
        e = hipEventCreate(&c->ev_stop);
    if (e != hipSuccess) {
        c->last_hip = e;
        st = SIEVE_EDEVICE;
    }
    if (st == SIEVE_OK)
        st = sv::engine_init(c, c->batch);
    if (st == SIEVE_OK)
        st = sv::noalloc_setup(c);
    if (st == SIEVE_OK)
        st = sv::ensure_primes(c, sv::kDefaultPrimeLimit);
    if (st != SIEVE_OK) {
        sieve_destroy(c);
        return st;
    }
    *out = c;
    return SIEVE_OK;
}

int sieve_destroy(sieve_ctx *c)
{
    if (!c)
        return SIEVE_OK;
    (void)hipSetDevice(c->device);
    if (c->stream)
        (void)hipStreamSynchronize(c->stream);
    // asynchronous calls on the caller's streams may still read the prime
    // table, their counter slot and the bucket pool
    for (int i = 0; i < sieve_ctx::kSlots; ++i)
        if (c->slot_used[i] && c->slot_done[i])
            (void)hipEventSynchronize(c->slot_done[i]);
    sv::engine_free(c->batch);
    for (sv::DevBuf *b : {&c->b_buckets, &c->b_bcount})
        if (b->p)
            (void)hipFree(b->p);
    if (c->d_primes)
        (void)hipFree(c->d_primes);
    if (c->d_inv)
        (void)hipFree(c->d_inv);
    if (c->d_ctr)
        (void)hipFree(c->d_ctr);
    for (int i = 0; i < sieve_ctx::kSlots; ++i)
        if (c->slot_done[i])
            (void)hipEventDestroy(c->slot_done[i]);
    if (c->h_ctr)
        (void)hipHostFree(c->h_ctr);
    if (c->ev_start)
        (void)hipEventDestroy(c->ev_start);
    if (c->ev_stop)
        (void)hipEventDestroy(c->ev_stop);
    if (c->stream)
        (void)hipStreamDestroy(c->stream);
    delete c;
    return SIEVE_OK;
}

int sieve_last_hip_error(const sieve_ctx *c)
{
    return c ? c->last_hip : 0;
}

int sieve_set_timing(sieve_ctx *c, int on)
{
    if (!c)
        return SIEVE_EINVAL;
    c->timing = on != 0;
    if (!c->timing)
        c->ev_valid = false;
    return SIEVE_OK;
}

int sieve_last_kernel_ms(sieve_ctx *c, double *ms)
{
    if (!c || !ms || !c->ev_valid)
        return SIEVE_EINVAL;
    SV_HIP_TRY(c, hipSetDevice(c->device));
    SV_HIP_TRY(c, hipEventSynchronize(c->ev_stop));
    float f = 0.f;
    SV_HIP_TRY(c, hipEventElapsedTime(&f, c->ev_start, c->ev_stop));
    *ms = f;
    return SIEVE_OK;
}

int sieve_get_tuning(const sieve_ctx *c, sieve_tuning *out)
{
    if (!c || !out)
        return SIEVE_EINVAL;
    *out = c->tuning;
    return SIEVE_OK;
}

int sieve_set_tuning(sieve_ctx *c, const sieve_tuning *t)
{
    if (!c || !t)
        return SIEVE_EINVAL;
    if (int st = sv::validate_tuning(*t, c->lds_max))
        return st;
    c->tuning = *t;
    return SIEVE_OK;
}

int sieve_base_primes(sieve_ctx *c, uint64_t limit, uint32_t *out, uint64_t cap, uint64_t *n_out)
{
    if (!c || !n_out)
        return SIEVE_EINVAL;
    if (limit > sv::kMaxPrimeLimit)
        return SIEVE_ERANGE;
    SV_HIP_TRY(c, hipSetDevice(c->device));
    if (int st = sv::ensure_primes(c, limit))
        return st;
    const auto &v = c->h_primes;
    const uint64_t n_odd = static_cast<uint64_t>(std::upper_bound(v.begin(), v.end(), limit) - v.begin());
    const uint64_t n = limit >= 2 ? n_odd + 1 : 0;
    if (!out || cap == 0) {
        *n_out = n;
        return SIEVE_OK;
    }
    if (cap < n) {
        *n_out = n;
        return SIEVE_EBUFSZ;
    }
    if (n) {
        out[0] = 2;
        std::memcpy(out + 1, v.data(), n_odd * sizeof(uint32_t));
    }
    *n_out = n;
    return SIEVE_OK;
}

int sieve_range_count(sieve_ctx *c, uint64_t lo, uint64_t hi, uint64_t *pi_out, void *stream)
{
    if (!c || !pi_out || lo > hi)
        return SIEVE_EINVAL;
    if (hi > SIEVE_MAX_HI)
        return SIEVE_ERANGE;
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    return sv::run_range(c, lo, hi, nullptr, pi_out, s);
}

int sieve_range_bitmap(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, uint64_t n_words,
                       uint64_t *pi_out, void *stream)
{
    if (!c || lo > hi)
        return SIEVE_EINVAL;
    if (hi > SIEVE_MAX_HI)
        return SIEVE_ERANGE;
    const uint64_t need = sieve_bitmap_words(lo, hi);
    if (need && !d_words)
        return SIEVE_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_words) % 4 != 0)
        return SIEVE_EINVAL;
    if (n_words < need)
        return SIEVE_EBUFSZ;
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    return sv::run_range(c, lo, hi, d_words, pi_out, s);
}

int sieve_batch(sieve_ctx *c, const sieve_interval *iv, uint32_t n, uint32_t *d_words,
                uint64_t total_words, uint64_t *pi_out, void *stream)
{
    if (!c || (n && (!iv || !pi_out)))
        return SIEVE_EINVAL;
    if (reinterpret_cast<uintptr_t>(d_words) % 4 != 0)
        return SIEVE_EINVAL;
    if (n == 0)
        return SIEVE_OK;
    if (int st = sv::engine_stage(c, c->batch, iv, n, d_words, total_words))
        return st;
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    if (int st = sv::engine_launch(c, c->batch, d_words, s, c->timing))
        return st;
    SV_HIP_TRY(c, hipEventSynchronize(c->batch.done));
    c->batch.pending = false;
    const unsigned long long *h_counts = sv::counts_host(c->batch);
    for (uint32_t i = 0; i < n; ++i)
        pi_out[i] = h_counts[i] + ((iv[i].lo <= 2 && 2 < iv[i].hi) ? 1 : 0);
    return SIEVE_OK;
}

int sieve_autotune(sieve_ctx *c, const sieve_interval *iv, uint32_t n, uint32_t flags, sieve_tuning *best,
                   double *best_ms)
{
    if (!c || !iv || n == 0 || !best)
        return SIEVE_EINVAL;
    uint64_t max_hi = 0, words = 0;
    for (uint32_t i = 0; i < n; ++i) {
        if (iv[i].lo > iv[i].hi)
            return SIEVE_EINVAL;
        if (iv[i].hi > SIEVE_MAX_HI)
            return SIEVE_ERANGE;
        max_hi = std::max(max_hi, iv[i].hi);
        words += sieve_bitmap_words(iv[i].lo, iv[i].hi);
    }
    int decade = 0;
    for (uint64_t x = max_hi; x >= 10; x /= 10)
        ++decade;
    int lg = 0;
    for (uint64_t x = words; x > 1; x >>= 1)
        ++lg;
    const auto key = std::make_tuple(n > 1 ? 1 : 0, decade, lg);
    auto hit = c->tune_cache.find(key);
    if (hit != c->tune_cache.end() && !(flags & SIEVE_TUNE_FORCE)) {
        *best = hit->second.first;
        if (best_ms)
            *best_ms = hit->second.second;
        if (flags & SIEVE_TUNE_APPLY)
            c->tuning = *best;
        return SIEVE_OK;
    }
    // The automatic plan first (so the answer is never slower than what the
    // context does untuned), then segment sizes with the workgroup size
    // measured best for each on the count of [2, 10^10), times three
    // dense/sparse bounds.
    struct SegChoice {
        uint32_t seg_bits, threads;
    };
    const SegChoice segs[] = {{1u << 17, 512}, {1u << 18, 512}, {1u << 19, 1024}, {sv::kWideSegWords * 32, 1024}};
    const uint32_t dense_div[] = {1024, 512, 256};
    const sieve_tuning saved = c->tuning;
    std::vector<sieve_tuning> cands;
    {
        sieve_tuning t = saved;
        t.seg_bits = 0;
        t.block_threads = 0;
        t.dense_limit = 0;
        cands.push_back(t);
    }
    for (const SegChoice &sc : segs) {
        if (sc.seg_bits / 32 > sv::max_seg_words(c->lds_max))
            continue;
        for (uint32_t dd : dense_div) {
            sieve_tuning t = saved;
            t.seg_bits = sc.seg_bits;
            t.block_threads = sc.threads;
            t.dense_limit = std::max(sc.seg_bits / dd, sv::kFirstMarkedPrime);
            cands.push_back(t);
        }
    }
    // A batch is timed as the caller will run it: intervals that want their
    // bitmap write it, into a scratch buffer of the batch's extent.
    uint64_t extent = 0;
    for (uint32_t i = 0; i < n && n > 1; ++i)
        if (iv[i].flags & SIEVE_WANT_BITMAP)
            extent = std::max(extent, iv[i].word_offset + sieve_bitmap_words(iv[i].lo, iv[i].hi));
    uint32_t *d_scratch = nullptr;
    if (extent) {
        SV_HIP_TRY(c, hipSetDevice(c->device));
        const hipError_t e = hipMalloc(&d_scratch, extent * sizeof(uint32_t));
        if (e != hipSuccess) {
            c->last_hip = e;
            return SIEVE_ENOMEM;
        }
    }
    const bool saved_timing = c->timing;
    c->timing = true;  // candidates are ranked by their kernel times
    sieve_tuning win{};
    double win_ms = 1e300;
    int st = SIEVE_OK;
    auto time_it = [&](const sieve_tuning &t) {
        c->tuning = t;
        double ms = 1e300;
        for (int rep = 0; rep < 3 && st == SIEVE_OK; ++rep) {
            if (n == 1) {
                uint64_t pi = 0;
                st = sv::run_range(c, iv[0].lo, iv[0].hi, nullptr, &pi, c->stream);
            } else {
                std::vector<uint64_t> pi(n);
                st = sieve_batch(c, iv, n, d_scratch, extent, pi.data(), nullptr);
            }
            double k = 0;
            if (st == SIEVE_OK && rep > 0 && sieve_last_kernel_ms(c, &k) == SIEVE_OK)
                ms = std::min(ms, k);  // the first run is a warm-up
        }
        if (st == SIEVE_OK && ms < win_ms) {
            win_ms = ms;
            win = t;
        }
    };
    for (const sieve_tuning &t : cands) {
        time_it(t);
        if (st != SIEVE_OK)
            break;
    }
    // Refine the winner: fewer resident workgroups per CU, and for a single
    // range that uses hit buckets, a higher large-prime threshold or none.
    std::vector<sieve_tuning> refine;
    if (st == SIEVE_OK) {
        for (uint32_t w : {1u, 2u}) {
            sieve_tuning t = win;
            t.wg_per_cu = w;
            refine.push_back(t);
        }
        sieve_plan_info pl{};
        if (n == 1 && sv::make_plan(iv[0].lo, iv[0].hi, &win, c->n_cu, c->lds_max, &pl) == SIEVE_OK &&
            pl.bucket_limit) {
            for (uint32_t f : {2u, 4u}) {
                sieve_tuning t = win;
                t.bucket_limit = static_cast<uint32_t>(std::min<uint64_t>(uint64_t(f) * pl.seg_bits, 0xfffffffeull));
                refine.push_back(t);
            }
            sieve_tuning t = win;
            t.bucket_limit = 0xffffffffu;  // never
            refine.push_back(t);
        }
    }
    for (const sieve_tuning &t : refine) {
        time_it(t);
        if (st != SIEVE_OK)
            break;
    }
    if (d_scratch) {
        (void)hipDeviceSynchronize();
        (void)hipFree(d_scratch);
    }
    c->tuning = saved;
    c->timing = saved_timing;
    if (!saved_timing)
        c->ev_valid = false;
    if (st != SIEVE_OK)
        return st;
    c->tune_cache[key] = {win, win_ms};
    *best = win;
    if (best_ms)
        *best_ms = win_ms;
    if (flags & SIEVE_TUNE_APPLY)
        c->tuning = win;
    return SIEVE_OK;
}

}  // extern "C"
