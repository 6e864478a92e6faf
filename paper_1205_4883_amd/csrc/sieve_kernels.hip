// HIP kernels of the exact range sieve for gfx950 (CDNA4, wave64).
//
// Each workgroup owns one segment of the odd-only bitmap at a time and keeps
// it in LDS (1 bit per odd integer, 1 = composite while marking).  The
// paper's per-node block of integers (Section 3.1, Eq. 3) becomes this
// segment; its crossing-off of the multiples of each prime (Section 3.1) is
// done in three stages:
//   1. pre-sieve: the multiples of 3..31 are ORed in from three periodic
//      bit patterns held in LDS (products 3*5*7*11*13, 17*19*23, 29*31),
//      one funnel shift per pattern per word, no atomics;
//   2. dense primes (37 <= p < dense_limit): one wavefront per prime.  Only
//      the multiples p*m with m prime to 15 are crossed off (3 | m or 5 | m
//      is already covered by the pre-sieve); over the odd m these form 256
//      classes modulo 480 odd steps, four per lane.  480*p bits is a whole
//      number of words (15p), so a class's bit inside its word never changes
//      and its word moves by 15p per mark: one LDS atomic OR and one add;
//   3. sparse primes: one lane per prime walks the multiples p*m with m
//      prime to 15 (a wheel of period 30, gaps 6,4,2,4,2,4,6,2), so 8 of
//      every 15 odd multiples are visited.  Those not carried from the
//      previous segment are handed out 64 at a time to the wavefronts as
//      they come free.
// Then every thread counts the unmarked bits of its words (popcount plus a
// wavefront shuffle reduction) and, for bitmap output, stores them to HBM.
//
// Crossing off starts at max(p*p, first odd multiple in the segment), so a
// base prime never marks itself; the pre-sieve does mark 3..31 themselves and
// leaves 1 unmarked, which the first word of a range corrects.
//
// LDS bank behaviour on gfx950 (32 banks of 4 bytes; each 32-lane half of a
// wave is served separately) sets the cost of the scattered atomic ORs.  The
// wheel cuts their number; the fixed-bit lane layout keeps the VALU work per
// dense mark at one add, and a per-prime choice of which classes share a
// half-wavefront spreads the dense marks over the banks.  A segment holds up
// to 19,456 words, the most with which two 1024-thread workgroups still fit
// in a CU's 160 KiB of LDS.
#include <atomic>

#include "dense_layout.h"
#include "sieve_internal.h"

namespace sv {
namespace {

constexpr uint32_t kLA = 3u * 5u * 7u * 11u * 13u;  // 15015
constexpr uint32_t kLB = 17u * 19u * 23u;           // 7429
constexpr uint32_t kLC = 29u * 31u;                 // 899
// The pre-sieve fills a segment in runs of up to kRun consecutive words per
// thread.  kRun is odd, and so is every run length used, so that the runs of
// a half-wavefront's 32 lanes start on 32 distinct LDS banks.
constexpr uint32_t kRun = 19;
// A table of period L holds the words k <= (L - 1) / 32 + kRun: enough for a
// run of kRun words starting at any phase j < L (word k of the run is a
// funnel shift of table words (j >> 5) + k and (j >> 5) + k + 1).
constexpr uint32_t kWA = (kLA - 1) / 32 + kRun + 1;  // 489
constexpr uint32_t kWB = (kLB - 1) / 32 + kRun + 1;  // 252
constexpr uint32_t kWC = (kLC - 1) / 32 + kRun + 1;  // 48
static_assert(kWA + kWB + kWC <= kTableWords, "pre-sieve tables exceed their LDS area");

// Odd residues r mod 30 prime to 15, as a bit mask.
constexpr uint32_t kWheelMask = (1u << 1) | (1u << 7) | (1u << 11) | (1u << 13) | (1u << 17) |
                                (1u << 19) | (1u << 23) | (1u << 29);
// Gaps between consecutive such residues, in odd steps (2 each), starting
// after residue 1: 3,2,1,2,1,2,3,1 as 2-bit fields, repeated twice so that a
// 2-bit rotation of the 32-bit word walks the cycle.
constexpr uint32_t kWheelGaps16 = 3u | (2u << 2) | (1u << 4) | (2u << 6) | (1u << 8) | (2u << 10) |
                                  (3u << 12) | (1u << 14);
constexpr uint32_t kWheelGaps = kWheelGaps16 | (kWheelGaps16 << 16);

__device__ __forceinline__ void lds_or(uint32_t *word, uint32_t mask)
{
    __hip_atomic_fetch_or(word, mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// The three pre-sieve tables, computed at compile time.  Bit b of a table's
// word k stands for the odd integer 2(32k + b) + 1 and is set when one of
// the group's primes divides it.
struct PresieveTables {
    uint32_t w[kTableWords];
};

constexpr uint32_t table_word(uint32_t k, const uint32_t *ps, int np)
{
    uint32_t m = 0;
    for (uint32_t b = 0; b < 32; ++b) {
        const uint32_t odd = 2 * (32 * k + b) + 1;
        for (int i = 0; i < np; ++i)
            if (odd % ps[i] == 0)
                m |= 1u << b;
    }
    return m;
}

constexpr PresieveTables make_tables()
{
    constexpr uint32_t pa[5] = {3, 5, 7, 11, 13};
    constexpr uint32_t pb[3] = {17, 19, 23};
    constexpr uint32_t pc[2] = {29, 31};
    PresieveTables t{};
    for (uint32_t k = 0; k < kWA; ++k)
        t.w[k] = table_word(k, pa, 5);
    for (uint32_t k = 0; k < kWB; ++k)
        t.w[kWA + k] = table_word(k, pb, 3);
    for (uint32_t k = 0; k < kWC; ++k)
        t.w[kWA + kWB + k] = table_word(k, pc, 2);
    return t;
}

__constant__ PresieveTables kTables = make_tables();

// Per dense prime, the lane layout of its wheel classes (see mark_dense).
struct DenseStrides {
    uint8_t u[kDenseStrideCount];
};

constexpr DenseStrides make_dense_strides()
{
    DenseStrides d{};
    for (uint32_t i = 0; i < kDenseStrideCount; ++i)
        d.u[i] = kDenseStride[i];
    return d;
}

__constant__ DenseStrides kDenseStrides = make_dense_strides();
static_assert(kFirstMarkedPrime == 37, "kDenseStride is indexed from the prime 37");

// Copy the tables into the workgroup's LDS (visible after its next barrier).
__device__ __forceinline__ void build_tables(uint32_t *tabs)
{
    for (uint32_t k = threadIdx.x; k < kTableWords; k += blockDim.x)
        tabs[k] = kTables.w[k];
}

// The first odd multiple m0*p of p with m0*p >= n0 and m0 >= p (crossing off
// starts at p*p), for the segment whose bit 0 is the odd integer n0.
//   off: its bit offset in the segment (at least lim_bits when past the
//        segment);
//   m30: m0 mod 30.
// nf = n0 as a double (exact: n0 < 2^53) and inv = 1/p rounded to double.
// floor(nf * inv) is within one of floor(n0 / p) (the product's relative
// error is below 2^-52 and n0 / p < 2^48), and the remainder n0 - q*p is an
// integer below 2^27 in magnitude, which an fma yields exactly; one
// correction step then makes q exact.
struct Start {
    uint32_t off;
    uint32_t m30;
};

__device__ __forceinline__ Start first_multiple(uint64_t n0, double nf, uint32_t p, double inv,
                                                uint32_t lim_bits)
{
    const double pf = static_cast<double>(p);
    double q = floor(nf * inv);
    double r = fma(-q, pf, nf);
    if (r < 0.0) {
        r += pf;
        q -= 1.0;
    } else if (r >= pf) {
        r -= pf;
        q += 1.0;
    }
    // k = ceil(n0 / p): the first multiplier with k*p >= n0
    uint32_t d = 0;  // k*p - n0
    if (r > 0.0) {
        d = p - static_cast<uint32_t>(r);
        q += 1.0;
    }
    const double t = floor(q * (1.0 / 30.0));
    int32_t k30 = static_cast<int32_t>(fma(-t, 30.0, q));  // exact, within one period of [0, 30)
    if (k30 < 0)
        k30 += 30;
    else if (k30 >= 30)
        k30 -= 30;
    if ((k30 & 1) == 0) {  // n0 is odd, so an even k gives an even multiple: take the next
        d += p;
        k30 += 1;
    }
    Start s{d >> 1, static_cast<uint32_t>(k30)};
    if (pf * pf > nf) {  // p*p lies past n0 (both exact in double): start there, m0 = p
        const uint64_t o2 = (static_cast<uint64_t>(p) * p - n0) >> 1;
        s.off = o2 < lim_bits ? static_cast<uint32_t>(o2) : lim_bits;
        s.m30 = p % 30u;
    }
    return s;
}

// Step from the odd multiple at bit offset o (multiplier m, m mod 30 = m30)
// to the first one whose multiplier is prime to 15 (at most two odd steps);
// returns the multiplier's position in the cycle of the eight wheel
// residues.
__device__ __forceinline__ uint32_t wheel_start(uint32_t p, uint32_t &o, uint32_t m30)
{
    while (((kWheelMask >> m30) & 1u) == 0) {
        m30 += 2;
        o += p;
    }
    return __popc(kWheelMask & ((1u << m30) - 1u)) & 7u;
}

// Dense marking of one prime by a whole wavefront.  Only the odd multiples
// p*m with m prime to 15 are crossed off (3 | m or 5 | m is already covered
// by the pre-sieve).  Counting odd multiples i = 0, 1, ... from the first
// such m, the kept i repeat with period 15 (8 per period), so over 480 odd
// steps there are 256 kept classes; the k-th of them (k = 0..255) is
// 15 (k / 8) + (the sum of the first k mod 8 gaps of the rotated cycle).
// Lane l takes in slot j = 0..3 the class with k = u (l + 64 j) mod 256:
// u is odd, so the 64 x 4 (lane, slot) pairs take every class once, and a
// lane's four classes lie 120 odd steps apart in some order.  480*p bits is
// a whole number of words (15p), so each class keeps a fixed bit and moves by
// 15p words per mark: one LDS atomic OR and one add.  u is chosen per prime
// (kDenseStrides) so that the 32 lanes of each half-wavefront spread over
// the LDS banks.  The largest class (fixed by the cycle alone) drives the
// loop (a scalar), and each class needs at most one guarded mark after it.
__device__ __forceinline__ void mark_dense(uint32_t *seg, uint32_t sw, uint32_t p, uint32_t s,
                                           uint32_t m30, uint32_t lane, uint32_t u)
{
    uint32_t o = s;
    const uint32_t idx = wheel_start(p, o, m30);
    const uint32_t g = __builtin_amdgcn_alignbit(kWheelGaps, kWheelGaps, 2 * idx);
    const uint32_t k0 = (u * lane) & 255u;
    const uint32_t first = g & ((1u << (2 * (k0 & 7))) - 1);
    const uint32_t e = __popc(first & 0x5555u) + 2 * __popc(first & 0xaaaau);  // k mod 8 = k0 mod 8
    const uint32_t ku = 64u * u;
    const uint32_t k1 = (k0 + ku) & 255u, k2 = (k0 + 2 * ku) & 255u, k3 = (k0 + 3 * ku) & 255u;
    const uint32_t c63 = 105 + 15 - ((g >> 14) & 3);  // the eight gaps sum to 15
    const uint32_t q = 120 * p;                       // odd steps between a lane's classes, in bits
    // dense primes are below 2^20 and classes below 480: full-rate 24-bit products
    const uint32_t x0 = o + __umul24(15 * (k0 >> 3) + e, p);
    const uint32_t x1 = o + __umul24(15 * (k1 >> 3) + e, p);
    const uint32_t x2 = o + __umul24(15 * (k2 >> 3) + e, p);
    const uint32_t x3 = o + __umul24(15 * (k3 >> 3) + e, p);
    uint32_t *p0 = seg + (x0 >> 5);
    uint32_t *p1 = seg + (x1 >> 5);
    uint32_t *p2 = seg + (x2 >> 5);
    uint32_t *p3 = seg + (x3 >> 5);
    const uint32_t m0 = 1u << (x0 & 31), m1 = 1u << (x1 & 31), m2 = 1u << (x2 & 31), m3 = 1u << (x3 & 31);
    const uint32_t step = 15 * p;
    for (uint32_t top = (o + c63 * p + 3 * q) >> 5; top < sw; top += step) {
        lds_or(p0, m0);
        lds_or(p1, m1);
        lds_or(p2, m2);
        lds_or(p3, m3);
        p0 += step;
        p1 += step;
        p2 += step;
        p3 += step;
    }
    uint32_t *const end = seg + sw;
    if (p0 < end)
        lds_or(p0, m0);
    if (p1 < end)
        lds_or(p1, m1);
    if (p2 < end)
        lds_or(p2, m2);
    if (p3 < end)
        lds_or(p3, m3);
}

// Sparse marking of one prime by one lane: the multiples p*m with m prime to
// 15 from bit offset o (whose multiplier sits at wheel position idx) up to
// lim_bits.  While a whole turn of the wheel (15 odd steps, 15p bits, 8
// marks) fits, the eight offsets of a turn are computed once and a mark costs
// one add plus the address and mask; only lanes whose prime is small enough
// build them, so a wavefront of large primes (a few marks per segment, the
// common case in batches near 1e12) skips the table.  The rest of the last
// turn is walked mark by mark along the rotated gaps.  Returns the offset of
// the first multiple left unmarked (at or past lim_bits) and sets idx to its
// wheel position, so that the next segment can continue from there.
// kSmall: p < 2^24, so the offsets are full-rate 24-bit products.
template <bool kSmall>
__device__ __forceinline__ uint32_t mark_wheel(uint32_t *seg, uint32_t lim_bits, uint32_t p, uint32_t o,
                                               uint32_t &idx)
{
    const uint32_t g = __builtin_amdgcn_alignbit(kWheelGaps, kWheelGaps, 2 * idx);
    uint32_t base = o;
    // the seven offsets after a turn's first multiple are at most 14p
    if (base + (kSmall ? __umul24(14u, p) : 14 * p) < lim_bits) {
        uint32_t d[8];
        d[0] = 0;
        uint32_t cum = 0;  // odd steps from the turn's first multiple
#pragma unroll
        for (int j = 1; j < 8; ++j) {
            cum += (g >> (2 * (j - 1))) & 3u;
            d[j] = kSmall ? __umul24(cum, p) : cum * p;
        }
        const uint32_t turn = kSmall ? __umul24(15u, p) : 15 * p;
        do {
#pragma unroll
            for (int j = 0; j < 8; ++j) {
                const uint32_t x = base + d[j];
                lds_or(seg + (x >> 5), 1u << (x & 31));
            }
            base += turn;
        } while (base + d[7] < lim_bits);
    }
    // at most one turn is left: base sits at wheel position idx again
    uint32_t s = 0;
    while (base < lim_bits) {
        lds_or(seg + (base >> 5), 1u << (base & 31));
        const uint32_t gap = (g >> (2 * s)) & 3u;
        base += kSmall ? __umul24(gap, p) : gap * p;
        ++s;
    }
    idx = (idx + s) & 7u;
    return base;
}

// The first word of a range: 1 is not prime; 3..31 are primes that the
// pre-sieve crossed off.  v has 1 = prime.
__device__ __forceinline__ uint32_t fix_first_word(uint32_t v, uint64_t first_odd)
{
    if (first_odd > 31)
        return v;
    if (first_odd == 1)
        v &= ~1u;
    const uint32_t f = static_cast<uint32_t>(first_odd);
    for (uint32_t p = 3; p <= 31; p += 2) {
        const bool prime = p != 9 && p != 15 && p != 21 && p != 25 && p != 27;
        if (prime && p >= f)
            v |= 1u << ((p - f) >> 1);
    }
    return v;
}

__device__ __forceinline__ uint32_t wave_sum(uint32_t v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

__device__ __forceinline__ unsigned long long wave_sum64(unsigned long long v)
{
    for (int off = 32; off > 0; off >>= 1)
        v += __shfl_xor(v, off, 64);
    return v;
}

constexpr uint32_t kNoItem = 0xffffffffu;

// The next work item of a launch, for thread 0 of a workgroup.  An atomic
// add on queue q's counter hands out items q, q + kQueues, q + 2 kQueues, ...
// Once q runs dry, all the counters are read together (independent loads,
// one round trip) and the pop moves to a queue that still has items, rather
// than trying each queue in turn with an atomic of its own (eight serial
// device-scope round trips at the end of every workgroup).  Counters only
// grow, so each failed pop retires a queue and the loop ends.  Returns
// kNoItem when every queue is dry.
__device__ __forceinline__ uint32_t pop_item(uint32_t *counters, uint32_t &q, uint32_t n_items)
{
    for (;;) {
        const uint32_t k = atomicAdd(counters + q * kLineWords, 1u);
        const uint64_t item = static_cast<uint64_t>(k) * kQueues + q;
        if (item < n_items)
            return static_cast<uint32_t>(item);
        uint32_t seen[kQueues];
#pragma unroll
        for (uint32_t j = 0; j < kQueues; ++j)
            seen[j] = __hip_atomic_load(counters + j * kLineWords, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        uint32_t next = kQueues;
#pragma unroll
        for (uint32_t d = kQueues - 1; d >= 1; --d) {  // nearest after q wins
            const uint32_t j = (q + d) % kQueues;
            if (static_cast<uint64_t>(seen[j]) * kQueues + j < n_items)
                next = j;
        }
        if (next == kQueues)
            return kNoItem;
        q = next;
    }
}

// Work item for thread 0 of workgroup b on its pass `pass` (0, 1, ...):
// with no more items than workgroups each takes item b once, with no queue
// at all; otherwise pop_item.
__device__ __forceinline__ uint32_t next_item(uint32_t *counters, uint32_t &q, uint32_t n_items, uint32_t pass)
{
    if (n_items <= gridDim.x)
        return pass == 0 && blockIdx.x < n_items ? blockIdx.x : kNoItem;
    return pop_item(counters, q, n_items);
}

// Sum of every thread's v over the workgroup, valid in thread 0 (red: one
// LDS word per wavefront).
__device__ __forceinline__ unsigned long long wg_sum(unsigned long long v, unsigned long long *red)
{
    v = wave_sum64(v);
    if ((threadIdx.x & 63) == 0)
        red[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long total = 0;
    if (threadIdx.x == 0)
        for (uint32_t w = 0; w < (blockDim.x >> 6); ++w)
            total += red[w];
    return total;
}

// Where one segment of a range lies.
struct SegGeom {
    uint64_t w0;        // first word of the segment in the range
    uint64_t n0;        // odd integer of the segment's bit 0
    double nf;          // n0 as a double (exact: n0 < 2^53)
    uint32_t sw;        // words in the segment (the last one may be short)
    uint32_t lim_bits;  // sw * 32
};

__device__ __forceinline__ SegGeom seg_geom(uint64_t seg, uint32_t seg_words_max, uint64_t first_odd,
                                            uint64_t n_words)
{
    SegGeom g;
    g.w0 = seg * seg_words_max;
    const uint64_t left = n_words - g.w0;
    g.sw = left < seg_words_max ? static_cast<uint32_t>(left) : seg_words_max;
    g.lim_bits = g.sw * 32;
    g.n0 = first_odd + 64 * g.w0;
    g.nf = static_cast<double>(g.n0);
    return g;
}

// 1. pre-sieve.  Bit i of the segment is the odd integer 2x + 1 with
//    x = (n0 >> 1) + i; pattern phases are x mod L.  Each thread fills runs
//    of `run` consecutive words (odd, at most kRun): after the phases of the
//    run's first word, every further word costs one read and one funnel
//    shift per table, and a word store.  Consecutive lanes' runs lie `run`
//    words apart, so the stores of a half-wavefront hit 32 distinct banks.
//    kFull unrolls the run completely (fastest where registers allow; the
//    batch kernel, which holds more state per item, takes a shorter unroll
//    so that nothing spills).
template <bool kFull>
__device__ __forceinline__ void seg_presieve(const uint32_t *tabs, uint32_t *seg_lds, const SegGeom &g)
{
    const uint32_t nthreads = blockDim.x;
    const uint32_t run = min(((g.sw + nthreads - 1) / nthreads) | 1u, kRun);
    const uint64_t x0 = g.n0 >> 1;
    const uint32_t ra = static_cast<uint32_t>(x0 % kLA);
    const uint32_t rb = static_cast<uint32_t>(x0 % kLB);
    const uint32_t rc = static_cast<uint32_t>(x0 % kLC);
    for (uint32_t w0 = threadIdx.x * run; w0 < g.sw; w0 += nthreads * run) {
        // 32 * w0 < 2^20: the phases of word w0, each reduced once
        uint32_t ja = ra + (32 * w0) % kLA;
        ja = min(ja, ja - kLA);
        uint32_t jb = rb + (32 * w0) % kLB;
        jb = min(jb, jb - kLB);
        uint32_t jc = rc + (32 * w0) % kLC;
        jc = min(jc, jc - kLC);
        const uint32_t *ta = tabs + (ja >> 5);
        const uint32_t *tb = tabs + kWA + (jb >> 5);
        const uint32_t *tc = tabs + kWA + kWB + (jc >> 5);
        uint32_t *out = seg_lds + w0;
        uint32_t a = ta[0], b = tb[0], c = tc[0];
        const uint32_t n = min(run, g.sw - w0);  // the segment's last run may be cut short
        auto word = [&](uint32_t k) {
            const uint32_t a1 = ta[k + 1], b1 = tb[k + 1], c1 = tc[k + 1];
            out[k] = __builtin_amdgcn_alignbit(a1, a, ja) | __builtin_amdgcn_alignbit(b1, b, jb) |
                     __builtin_amdgcn_alignbit(c1, c, jc);
            a = a1;
            b = b1;
            c = c1;
        };
        if (kFull) {
#pragma unroll
            for (uint32_t k = 0; k < kRun; ++k)
                if (k < n)
                    word(k);
        } else {
#pragma unroll 4
            for (uint32_t k = 0; k < n; ++k)
                word(k);
        }
    }
}

// 2a. dense primes: one wavefront per prime.  Lane l of wave w computes the
//     start of prime r*64*nw + l*nw + w, so each wave gets an interleaved
//     share of the primes; the wave then marks its (up to) 64 primes one
//     after another.  The share is heaviest for wave 0 (the smallest prime
//     of every group of nw).  The order depends on the work item:
//     - kDensePlain (single segments of a range): waves 0..nw-1 in order;
//     - kDenseReversed (pairs of segments, and batch items): numbered from
//       the other end.  The carried sparse primes weigh most on the first
//       waves (a wave's lanes hold consecutive primes, the smallest in wave
//       0), so those waves get the lightest dense share ([2, 1e10) before
//       the change below: 0.647 -> 0.636 ms; single segments of a range lost
//       up to 6%; the 4096-interval batch, whose sparse primes are all
//       shared: 3.094 -> 3.065 ms);
//     - kDenseOldest (runs of three or more segments without hit buckets):
//       only waves 0..7 take dense primes, two per SIMD, numbered from the
//       other end.  Timed per wave, the waves a workgroup issues first run
//       fastest, and waves 8..15 then go straight to their carried and
//       shared sparse primes ([2, 1e10): 0.620 -> 0.607 ms, 10^10 integers
//       at 10^12: 1.589 -> 1.574 ms; four, six, ten or twelve dense waves
//       measured slower).  With hit buckets the reversed order is kept
//       (10^10 integers at 10^13: 2.53 -> 2.47 ms against this order).
enum DenseOrder : uint32_t { kDensePlain, kDenseReversed, kDenseOldest };
constexpr uint32_t kDenseOldestWaves = 8;

__device__ __forceinline__ void seg_dense(uint32_t *seg_lds, const SegGeom &g, const uint32_t *primes,
                                          const double *inv, uint32_t n_dense, DenseOrder order = kDensePlain)
{
    const uint32_t t = threadIdx.x;
    const uint32_t lane = t & 63;
    uint32_t nw = blockDim.x >> 6;
    uint32_t wave = t >> 6;
    if (order == kDenseOldest && nw >= kDenseOldestWaves) {
        if (wave >= kDenseOldestWaves)
            return;
        nw = kDenseOldestWaves;
    }
    if (order != kDensePlain)
        wave = nw - 1 - wave;
    for (uint32_t r0 = 0; r0 + wave < n_dense; r0 += 64 * nw) {
        const uint32_t i = r0 + lane * nw + wave;
        uint32_t p = 0, s0 = 0, m30 = 0, u = 1;
        if (i < n_dense) {
            p = primes[i];
            const Start st = first_multiple(g.n0, g.nf, p, inv[i], g.lim_bits);
            s0 = st.off;
            m30 = st.m30;
            if (i < kDenseStrideCount)
                u = kDenseStrides.u[i];
        }
        const uint32_t cnt = min(64u, (n_dense - r0 - wave + nw - 1) / nw);
        for (uint32_t l = 0; l < cnt; ++l)
            mark_dense(seg_lds, g.sw, __builtin_amdgcn_readlane(p, l), __builtin_amdgcn_readlane(s0, l),
                       __builtin_amdgcn_readlane(m30, l), lane, __builtin_amdgcn_readlane(u, l));
    }
}

// Whether every marking prime is below 2^24 (the largest is the last).
__device__ __forceinline__ bool small_primes(const uint32_t *primes, uint32_t n_primes)
{
    return n_primes == 0 || primes[n_primes - 1] < (1u << 24);
}

// 2c. large primes: the segment's bucket of precomputed hits.
__device__ __forceinline__ void seg_buckets(uint32_t *seg_lds, uint64_t seg, const uint32_t *buckets,
                                            const uint32_t *bucket_count, uint32_t bucket_depth)
{
    const uint32_t nb = min(bucket_count[seg], bucket_depth);
    const uint32_t *bk = buckets + seg * bucket_depth;
    for (uint32_t e = threadIdx.x; e < nb; e += blockDim.x) {
        const uint32_t b = bk[e];
        lds_or(seg_lds + (b >> 5), 1u << (b & 31));
    }
}

// 3. count (and store) the unmarked bits; returns this thread's count.  The
//    marking must be complete (a __syncthreads after it).  Only the range's
//    first word (small primes, 1) and last word (tail bits) need fixing;
//    both are patched in LDS by one thread before the sweep.
template <bool kWrite>
__device__ __forceinline__ uint32_t seg_count(uint32_t *seg_lds, const SegGeom &g, uint64_t first_odd,
                                              uint64_t nbits, uint64_t n_words, uint32_t *out)
{
    const uint32_t t = threadIdx.x;
    const uint32_t tail = static_cast<uint32_t>(nbits & 31);
    const bool first = g.w0 == 0, last = tail && g.w0 + g.sw == n_words;
    if (first || last) {  // uniform over the workgroup
        if (t == 0) {
            if (first)
                seg_lds[0] = ~fix_first_word(~seg_lds[0], first_odd);
            if (last)
                seg_lds[g.sw - 1] |= ~((1u << tail) - 1);
        }
        __syncthreads();
    }
    uint32_t c = 0;
    uint32_t *o = kWrite ? out + g.w0 : nullptr;
    for (uint32_t w = t; w < g.sw; w += blockDim.x) {
        const uint32_t v = ~seg_lds[w];
        c += __popc(v);
        if (kWrite)
            o[w] = v;
    }
    return c;
}

// Thread 0 of each workgroup, as it leaves, with the workgroup's count.  The
// count and the "finished" tally travel in one read-modify-write each, so no
// fence is needed: workgroup b adds (count << 16) | 1 to count line
// b mod kQueues; the workgroup whose add completes its line (the returned
// tally shows it was the line's last) adds (line total << 8) | 1 to the grid
// word; and the one that completes the grid word holds the launch's total in
// the returned value.  It then returns the counter block to zero for the
// next launch (keeping the running total in the grid word between the
// launches of one call) and, on the call's last launch, publishes the total.
__device__ void finish_launch(const RangeArgs &r, unsigned long long wg_count)
{
    const uint32_t grid = gridDim.x;
    const uint32_t q = blockIdx.x % kQueues;
    const uint32_t in_line = grid / kQueues + (q < grid % kQueues ? 1u : 0u);
    const uint32_t lines = grid < kQueues ? grid : kQueues;
    auto *line = reinterpret_cast<unsigned long long *>(r.counters + (kQueues + q) * kLineWords);
    const unsigned long long old = atomicAdd(line, (wg_count << 16) | 1ull);
    if ((old & 0xffffu) + 1 != in_line)
        return;
    const unsigned long long line_total = (old >> 16) + wg_count;
    auto *all = reinterpret_cast<unsigned long long *>(r.counters + kDoneWord);
    const unsigned long long old2 = atomicAdd(all, (line_total << 8) | 1ull);
    if ((old2 & 0xffu) + 1 != lines)
        return;
    const unsigned long long total = (old2 >> 8) + line_total;
    // every workgroup has left: no pop or add on this block is still to come
    for (uint32_t k = 0; k < kQueues; ++k) {
        __hip_atomic_store(r.counters + k * kLineWords, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(reinterpret_cast<unsigned long long *>(r.counters + (kQueues + k) * kLineWords), 0ull,
                           __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __hip_atomic_store(all, r.last ? 0ull : total << 8, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    if (r.last && r.publish)
        *r.publish = total + r.publish_add;  // read after the stream (or the published word) says so
}

// 2b. sparse primes [i_begin, n_primes), one lane per prime, each start
//     computed afresh for this segment, shared out among the wavefronts as
//     they come free: a wave takes the next 64 primes (a lane each) from
//     the workgroup's LDS counter `units` (zero when the segment's marking
//     starts), so that waves whose other marking ended early take more.
template <bool kSmall>
__device__ __forceinline__ void seg_sparse_shared(uint32_t *seg, const SegGeom &g, const uint32_t *primes,
                                                  const double *inv, uint32_t i_begin, uint32_t n_primes,
                                                  uint32_t *units)
{
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t n_units = n_primes > i_begin ? (n_primes - i_begin + 63) / 64 : 0;
    if (n_units == 0)
        return;
    uint32_t w = 0;
    if (lane == 0)
        w = atomicAdd(units, 1u);
    w = __builtin_amdgcn_readfirstlane(w);
    while (w < n_units) {
        // take the next unit now, so that the atomic's trip through the
        // busy LDS queue overlaps this unit's marking
        uint32_t next = 0;
        if (lane == 0)
            next = atomicAdd(units, 1u);
        const uint32_t i = i_begin + w * 64 + lane;
        if (i < n_primes) {
            const uint32_t p = primes[i];
            const Start st = first_multiple(g.n0, g.nf, p, inv[i], g.lim_bits);
            uint32_t o = st.off;
            uint32_t idx = wheel_start(p, o, st.m30);
            (void)mark_wheel<kSmall>(seg, g.lim_bits, p, o, idx);
        }
        w = __builtin_amdgcn_readfirstlane(next);
    }
}

// Sieve segment `seg` of one range into LDS and emit its words; returns the
// number of primes among this thread's words.  tabs: the pre-sieve tables in
// LDS; seg_lds: seg_words_max words of LDS, which the caller may reuse after
// its next __syncthreads.  kSmall: every marking prime is below 2^24.
// units: the workgroup's LDS counter for the shared sparse primes, zero
// before the segment's first barrier (4096 seeded intervals in one batch:
// 3.12 -> 3.09 ms against a fixed split).
template <bool kWrite, bool kSmall>
__device__ uint32_t sieve_segment(const uint32_t *tabs, uint32_t *seg_lds, uint32_t seg_words_max,
                                  uint64_t seg, uint64_t first_odd, uint64_t nbits, uint64_t n_words,
                                  const uint32_t *primes, const double *inv, uint32_t n_dense,
                                  uint32_t n_primes, uint32_t *out, uint32_t *units)
{
    const SegGeom g = seg_geom(seg, seg_words_max, first_odd, n_words);
    seg_presieve<false>(tabs, seg_lds, g);
    __syncthreads();
    seg_dense(seg_lds, g, primes, inv, n_dense, kDenseReversed);
    seg_sparse_shared<kSmall>(seg_lds, g, primes, inv, n_dense, n_primes, units);
    __syncthreads();
    return seg_count<kWrite>(seg_lds, g, first_odd, nbits, n_words, out);
}

// Sparse primes whose next multiple a lane carries from one segment to the
// next, per thread; a carried state packs the offset (below kCarryCap) with
// the wheel position in the top three bits.
constexpr int kCarry = 4;
constexpr uint32_t kCarryCap = 1u << 28;
constexpr uint32_t kCarryNone = 0xffffffffu;

// The sparse primes of one segment (of a run): the first kCarry per lane
// continue from the multiple carried over from the previous segment (or
// start afresh on a run's first segment, k == 0).  The rest start afresh,
// shared out 64 at a time, a lane each, to the wavefronts as they come free
// from the workgroup's LDS counter `units` (zero at the segment's start):
// the waves whose fixed share (dense primes, carried primes) ends early
// take more, so fewer wait at the marking barrier.  (Timed per wave, the
// youngest waves of a workgroup, issued last, end their fixed share last;
// [2, 1e10): 0.634 -> 0.623 ms.)
template <bool kSmall>
__device__ __forceinline__ void sparse_phase(uint32_t *seg, const SegGeom &g, const PrimeArgs &pa, uint32_t t,
                                             uint32_t k, uint32_t carry_end, uint32_t (&carry)[kCarry],
                                             uint32_t *units)
{
#pragma unroll
    for (int j = 0; j < kCarry; ++j) {
        const uint32_t i = pa.n_dense + t + j * blockDim.x;
        if (i >= carry_end)
            break;
        const uint32_t p = pa.primes[i];
        uint32_t o, idx;
        if (k == 0 || carry[j] == kCarryNone) {
            const Start st = first_multiple(g.n0, g.nf, p, pa.inv[i], kCarryCap);
            o = st.off;
            if (o >= kCarryCap) {  // p*p lies far ahead: look again next segment
                carry[j] = kCarryNone;
                continue;
            }
            idx = wheel_start(p, o, st.m30);
        } else {
            o = carry[j] & (kCarryCap - 1);
            idx = carry[j] >> 29;
        }
        o = mark_wheel<kSmall>(seg, g.lim_bits, p, o, idx) - g.lim_bits;
        carry[j] = o < kCarryCap ? (idx << 29) | o : kCarryNone;
    }
    seg_sparse_shared<kSmall>(seg, g, pa.primes, pa.inv, carry_end, pa.n_primes, units);
}

// Resident workgroups pop work items from the launch's work queues (zero at
// launch) until every item is taken, so the grid size need not match the
// number of workgroups that fit on the device.  Items [0, n_chunks) are runs
// of `chunk` consecutive segments, the rest single segments (the tail, so
// that workgroups finish together).  Inside a run each lane carries the next
// multiple of its first kCarry sparse primes from segment to segment instead
// of dividing again.  Each workgroup adds its share of the count once, as it
// leaves.  The LDS segment is a static array of kSegMax words, so LDS
// addresses are compile-time offsets; a launch may use any seg_words <=
// kSegMax.  (Registers are capped so that eight waves fit per SIMD where LDS
// allows.)
template <uint32_t kSegMax, bool kWrite>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) range_kernel(
    RangeArgs r, PrimeArgs pa, uint32_t seg_words, uint32_t n_segments, uint32_t chunk, uint32_t n_chunks)
{
    __shared__ __align__(16) uint32_t lds[kTableWords + kSegMax];
    __shared__ uint32_t item_sh;
    __shared__ uint32_t units;
    __shared__ unsigned long long red[16];
    uint32_t *tabs = lds;
    uint32_t *seg = lds + kTableWords;
    build_tables(tabs);
    const uint32_t t = threadIdx.x;
    const uint32_t n_items = n_chunks + (n_segments - n_chunks * chunk);
    const uint32_t carry_end = min(pa.n_primes, pa.n_dense + kCarry * blockDim.x);
    const bool small = small_primes(pa.primes, pa.n_primes);
    uint32_t q = blockIdx.x % kQueues;
    unsigned long long acc = 0;
    uint32_t carry[kCarry];
    for (uint32_t pass = 0;; ++pass) {
        __syncthreads();  // tables built / the previous segment's LDS is free
        if (t == 0)
            item_sh = next_item(r.counters, q, n_items, pass);
        __syncthreads();
        const uint32_t item = item_sh;
        if (item == kNoItem)
            break;
        const uint64_t first = item < n_chunks ? static_cast<uint64_t>(item) * chunk
                                               : static_cast<uint64_t>(n_chunks) * chunk + (item - n_chunks);
        const uint32_t count = item < n_chunks ? chunk : 1;
        for (uint32_t k = 0; k < count; ++k) {
            if (k)
                __syncthreads();  // the previous segment's count has read the LDS
            const SegGeom g = seg_geom(first + k, seg_words, r.first_odd, r.n_words);
            if (t == 0)
                units = 0;  // no wave takes a unit before the barrier below
            seg_presieve<true>(tabs, seg, g);
            __syncthreads();
            seg_dense(seg, g, pa.primes, pa.inv, pa.n_dense,
                      count > 2 && !r.buckets ? kDenseOldest : count > 1 ? kDenseReversed : kDensePlain);
            if (small)
                sparse_phase<true>(seg, g, pa, t, k, carry_end, carry, &units);
            else
                sparse_phase<false>(seg, g, pa, t, k, carry_end, carry, &units);
            if (r.buckets)
                seg_buckets(seg, first + k, r.buckets, r.bucket_count, r.bucket_depth);
            __syncthreads();
            acc += seg_count<kWrite>(seg, g, r.first_odd, r.nbits, r.n_words, r.out);
        }
    }
    const unsigned long long wg_count = r.count ? wg_sum(acc, red) : 0;
    if (threadIdx.x == 0)
        finish_launch(r, wg_count);
}

// Persistent batch kernel: workgroups pop (interval, segment) items from the
// blob's work queues until every item is taken (hdr->n_items items).  Every
// workgroup leaves once all queues are dry, so the grid always drains.  Each
// item's count goes to item_counts[item] with a plain store (thread 0, at
// the next pop).  All sizes are read from device memory, so one captured
// graph serves batches of any size up to its buffers' capacity.
template <uint32_t kSegMax, bool kSmall>
__global__ void __launch_bounds__(1024) __attribute__((amdgpu_waves_per_eu(8, 8))) batch_kernel(
    BatchHeader *hdr, const uint32_t *primes, const double *inv, uint32_t *words,
    uint32_t *item_counts, uint32_t seg_words)
{
    __shared__ __align__(16) uint32_t lds[kTableWords + kSegMax];
    __shared__ uint32_t item_sh;
    __shared__ uint32_t units;
    __shared__ uint32_t red[16];
    uint32_t *tabs = lds;
    uint32_t *seg = lds + kTableWords;
    build_tables(tabs);
    const uint32_t n_items = hdr->n_items;
    char *blob = reinterpret_cast<char *>(hdr);
    uint32_t *counters = reinterpret_cast<uint32_t *>(blob + kBlobCounterOff);
    const BatchInterval *ivs = reinterpret_cast<const BatchInterval *>(blob + hdr->iv_off);
    const uint32_t *item_iv = reinterpret_cast<const uint32_t *>(blob + hdr->item_off);
    uint32_t q = blockIdx.x % kQueues;
    uint32_t prev = kNoItem;
    for (uint32_t pass = 0;; ++pass) {
        __syncthreads();  // red[] holds the previous item's wave counts; LDS is free
        if (threadIdx.x == 0) {
            if (prev != kNoItem) {
                uint32_t total = 0;
                for (uint32_t w = 0; w < (blockDim.x >> 6); ++w)
                    total += red[w];
                item_counts[prev] = total;
            }
            item_sh = next_item(counters, q, n_items, pass);
            units = 0;  // every wave has left the previous item's marking
        }
        __syncthreads();
        const uint32_t item = item_sh;
        if (item == kNoItem)
            break;
        const uint32_t k = item_iv[item];
        const BatchInterval iv = ivs[k];
        const uint64_t s = item - iv.seg_begin;
        uint32_t c;
        if (iv.word_offset != ~0ull)
            c = sieve_segment<true, kSmall>(tabs, seg, seg_words, s, iv.first_odd, iv.nbits, iv.n_words, primes, inv,
                                    iv.n_dense, iv.n_primes, words + iv.word_offset, &units);
        else
            c = sieve_segment<false, kSmall>(tabs, seg, seg_words, s, iv.first_odd, iv.nbits, iv.n_words, primes, inv,
                                     iv.n_dense, iv.n_primes, nullptr, &units);
        c = wave_sum(c);
        if ((threadIdx.x & 63) == 0)
            red[threadIdx.x >> 6] = c;
        prev = item;
    }
}

// Copies a batch's blob (header, work queues, interval table, work list)
// from the pinned host staging into device memory, with the work-queue
// counters cleared, so that a batch launch is kernels only: no runtime copy
// call (hipMemcpyAsync or a graph memcpy node).  The length is the header's
// blob_chunks, read once per wavefront from the host copy.
__global__ void __launch_bounds__(256) batch_stage_kernel(const uint4 *src, uint4 *dst)
{
    const uint32_t n = __builtin_amdgcn_readfirstlane(reinterpret_cast<const BatchHeader *>(src)->blob_chunks);
    constexpr uint32_t c0 = kBlobCounterOff / 16, c1 = kBlobIntervalOff / 16;
    static_assert(kBlobCounterOff % 16 == 0 && kBlobIntervalOff % 16 == 0, "blob regions are 16-byte chunks");
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        dst[i] = (i >= c0 && i < c1) ? make_uint4(0, 0, 0, 0) : src[i];
}

// counts[k] = the sum of item_counts over interval k's items, one wavefront
// per interval.
__global__ void __launch_bounds__(256) batch_reduce_kernel(const BatchHeader *hdr, const uint32_t *item_counts,
                                                           unsigned long long *counts)
{
    const uint32_t n = hdr->n_intervals;
    const uint32_t sw = hdr->seg_words;
    const BatchInterval *ivs =
        reinterpret_cast<const BatchInterval *>(reinterpret_cast<const char *>(hdr) + hdr->iv_off);
    const uint32_t lane = threadIdx.x & 63;
    const uint32_t waves = (gridDim.x * blockDim.x) >> 6;
    for (uint32_t k = (blockIdx.x * blockDim.x + threadIdx.x) >> 6; k < n; k += waves) {
        const BatchInterval iv = ivs[k];
        const uint64_t segs = (iv.n_words + sw - 1) / sw;
        unsigned long long c = 0;
        for (uint64_t j = lane; j < segs; j += 64)
            c += item_counts[iv.seg_begin + j];
        c = wave_sum64(c);
        if (lane == 0)
            counts[k] = c;
    }
}

// dst[0, n_words) = src[0, n_words), 16 bytes per thread and step, four
// loads in flight per thread (both 16-byte aligned).  The server returns
// bitmaps with it into its pinned host arena, mapped into the device, so
// that a copy is a kernel launch of its own in stream order on the lane
// instead of a runtime copy call (hipMemcpyAsync).
__global__ void __launch_bounds__(256) copy_words_kernel(const uint4 *src, uint4 *dst, uint64_t n_words)
{
    constexpr int kU = 4;
    const uint64_t n16 = n_words / 4;
    const uint64_t t = static_cast<uint64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    const uint64_t stride = static_cast<uint64_t>(gridDim.x) * blockDim.x;
    uint64_t i = t;
    for (; i + (kU - 1) * stride < n16; i += kU * stride) {
        uint4 v[kU];
#pragma unroll
        for (int k = 0; k < kU; ++k)
            v[k] = src[i + k * stride];
#pragma unroll
        for (int k = 0; k < kU; ++k)
            dst[i + k * stride] = v[k];
    }
    for (; i < n16; i += stride)
        dst[i] = src[i];
    if (t < n_words % 4)
        reinterpret_cast<uint32_t *>(dst)[4 * n16 + t] = reinterpret_cast<const uint32_t *>(src)[4 * n16 + t];
}

// Odd integers below 2^16 in one workgroup: bit i of bits[] is 2i + 1,
// 1 = composite.  For each odd p with p*p < 2^16 still unmarked, the threads
// cross off p*p, p*p + 2p, ... together; then the unmarked bits are compacted
// into the ascending list of odd primes.
__global__ void __launch_bounds__(1024) bootstrap_kernel(uint32_t *out, uint32_t *out_count)
{
    constexpr uint32_t kWords = kBootstrapLimit / 64;  // 1024
    __shared__ uint32_t bits[kWords];
    __shared__ uint32_t scan[kWords];
    const uint32_t t = threadIdx.x;
    for (uint32_t w = t; w < kWords; w += blockDim.x)
        bits[w] = (w == 0) ? 1u : 0u;  // 1 is not prime
    __syncthreads();
    for (uint32_t p = 3; p * p < kBootstrapLimit; p += 2) {
        const uint32_t i = p >> 1;
        const bool prime = ((bits[i >> 5] >> (i & 31)) & 1u) == 0;
        if (prime)
            for (uint32_t m = p * p + 2 * p * t; m < kBootstrapLimit; m += 2 * p * blockDim.x)
                lds_or(&bits[(m >> 1) >> 5], 1u << ((m >> 1) & 31));
        __syncthreads();
    }
    // exclusive scan of per-word prime counts (Hillis-Steele in LDS)
    for (uint32_t w = t; w < kWords; w += blockDim.x)
        scan[w] = __popc(~bits[w]);
    __syncthreads();
    for (uint32_t d = 1; d < kWords; d <<= 1) {
        uint32_t add[kWords / 256];
        uint32_t k = 0;
        for (uint32_t w = t; w < kWords; w += blockDim.x, ++k)
            add[k] = w >= d ? scan[w - d] : 0;
        __syncthreads();
        k = 0;
        for (uint32_t w = t; w < kWords; w += blockDim.x, ++k)
            scan[w] += add[k];
        __syncthreads();
    }
    for (uint32_t w = t; w < kWords; w += blockDim.x) {
        uint32_t v = ~bits[w];
        uint32_t pos = scan[w] - __popc(v);  // inclusive -> exclusive
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            out[pos++] = 2 * (32 * w + b) + 1;
        }
    }
    if (t == 0)
        *out_count = scan[kWords - 1];
}

// Compaction of a bitmap (1 = prime) into the integers its bits stand for.
constexpr uint32_t kCompactThreads = 256;
constexpr uint32_t kCompactPerThread = 16;
constexpr uint32_t kCompactChunk = kCompactThreads * kCompactPerThread;  // words per block

__global__ void __launch_bounds__(kCompactThreads) compact_count_kernel(const uint32_t *words,
                                                                        uint64_t n_words,
                                                                        uint32_t *block_sum)
{
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kCompactChunk;
    uint32_t c = 0;
    for (uint32_t k = threadIdx.x; k < kCompactChunk; k += kCompactThreads)
        if (base + k < n_words)
            c += __popc(words[base + k]);
    c = wave_sum(c);
    __shared__ uint32_t part[kCompactThreads / 64];
    if ((threadIdx.x & 63) == 0)
        part[threadIdx.x >> 6] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t s = 0;
        for (uint32_t i = 0; i < kCompactThreads / 64; ++i)
            s += part[i];
        block_sum[blockIdx.x] = s;
    }
}

// One workgroup: exclusive prefix sum of n block sums, in place; total to *total.
__global__ void __launch_bounds__(1024) compact_scan_kernel(uint32_t *block_sum, uint32_t n,
                                                            uint32_t *total)
{
    __shared__ uint32_t part[1024];
    const uint32_t t = threadIdx.x;
    const uint32_t per = (n + blockDim.x - 1) / blockDim.x;
    const uint32_t b = t * per;
    const uint32_t e = min(n, b + per);
    uint32_t s = 0;
    for (uint32_t i = b; i < e; ++i)
        s += block_sum[i];
    part[t] = s;
    __syncthreads();
    if (t == 0) {
        uint32_t run = 0;
        for (uint32_t i = 0; i < blockDim.x; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
        *total = run;
    }
    __syncthreads();
    uint32_t run = part[t];
    for (uint32_t i = b; i < e; ++i) {
        const uint32_t v = block_sum[i];
        block_sum[i] = run;
        run += v;
    }
}

__global__ void __launch_bounds__(kCompactThreads) compact_write_kernel(const uint32_t *words,
                                                                        uint64_t n_words,
                                                                        uint64_t first_odd,
                                                                        const uint32_t *block_off,
                                                                        uint32_t *out)
{
    __shared__ uint32_t part[kCompactThreads];
    const uint64_t base = static_cast<uint64_t>(blockIdx.x) * kCompactChunk +
                          static_cast<uint64_t>(threadIdx.x) * kCompactPerThread;
    uint32_t c = 0;
    for (uint32_t k = 0; k < kCompactPerThread; ++k)
        if (base + k < n_words)
            c += __popc(words[base + k]);
    part[threadIdx.x] = c;
    __syncthreads();
    if (threadIdx.x == 0) {
        uint32_t run = 0;
        for (uint32_t i = 0; i < kCompactThreads; ++i) {
            const uint32_t v = part[i];
            part[i] = run;
            run += v;
        }
    }
    __syncthreads();
    uint32_t pos = block_off[blockIdx.x] + part[threadIdx.x];
    for (uint32_t k = 0; k < kCompactPerThread; ++k) {
        if (base + k >= n_words)
            break;
        uint32_t v = words[base + k];
        while (v) {
            const uint32_t b = __builtin_ctz(v);
            v &= v - 1;
            out[pos++] = static_cast<uint32_t>(first_odd + 2 * (32 * (base + k) + b));
        }
    }
}

// Walk the wheel-30 multiples of one large prime over one chunk, calling
// hit(off) for each bit offset off < chunk_bits.
template <typename F>
__device__ __forceinline__ void walk_hits(uint64_t n0, uint32_t p, double inv, uint32_t chunk_bits, F hit)
{
    const Start st = first_multiple(n0, static_cast<double>(n0), p, inv, chunk_bits);
    uint32_t o = st.off;
    const uint32_t idx = wheel_start(p, o, st.m30);
    uint32_t g = __builtin_amdgcn_alignbit(kWheelGaps, kWheelGaps, 2 * idx);
    while (o < chunk_bits) {
        hit(o);
        o += (g & 3u) * p;
        g = __builtin_amdgcn_alignbit(g, g, 2);
    }
}

// The segment of a chunk that holds bit offset o, and o's offset in it.  A
// power-of-two segment (seg_log2 > 0) takes shifts.  Otherwise the float
// quotient o * (1 / seg_bits) is within one of the true one (o < 2^25 and the
// quotient below 33, so its relative error of a few 2^-24 cannot move it by
// a whole unit), and one correction step makes it exact.
__device__ __forceinline__ uint32_t seg_split(uint32_t o, uint32_t seg_bits, uint32_t seg_log2, float rcp,
                                              uint32_t &off)
{
    if (seg_log2) {
        off = o & (seg_bits - 1u);
        return o >> seg_log2;
    }
    uint32_t q = static_cast<uint32_t>(static_cast<float>(o) * rcp);
    uint32_t b = __umul24(q, seg_bits);  // q < 33, seg_bits < 2^24
    if (b > o) {
        --q;
        b -= seg_bits;
    } else if (o - b >= seg_bits) {
        ++q;
        b += seg_bits;
    }
    off = o - b;
    return q;
}

// One workgroup: a chunk of kBucketChunk segments (blockIdx.y) against 256
// large primes (blockIdx.x).  Two passes over the same hits: the first
// counts them per segment in LDS, then one global atomic per segment
// reserves room in its bucket, and the second writes each hit at its rank.
__global__ void __launch_bounds__(256) bucket_fill_kernel(const uint32_t *primes, const double *inv,
                                                          uint32_t n_large, uint64_t first_odd, uint32_t seg_bits,
                                                          uint32_t n_segs, uint32_t *buckets, uint32_t *bucket_count,
                                                          uint32_t depth, uint32_t *overflow)
{
    __shared__ uint32_t cnt[kBucketChunk];
    __shared__ uint32_t base[kBucketChunk];
    const uint32_t t = threadIdx.x;
    const uint32_t i = blockIdx.x * blockDim.x + t;
    const uint32_t seg0 = blockIdx.y * kBucketChunk;
    const uint32_t segs = min(kBucketChunk, n_segs - seg0);
    const uint32_t chunk_bits = segs * seg_bits;  // at most 32 x 622,592 < 2^25
    const uint64_t n0 = first_odd + 2 * static_cast<uint64_t>(seg0) * seg_bits;
    const uint32_t seg_log2 = (seg_bits & (seg_bits - 1u)) == 0 ? 31u - __builtin_clz(seg_bits) : 0u;
    const float rcp = 1.0f / static_cast<float>(seg_bits);
    if (t < kBucketChunk)
        cnt[t] = 0;
    __syncthreads();
    const bool live = i < n_large;
    const uint32_t p = live ? primes[i] : 0;
    const double pinv = live ? inv[i] : 0.0;
    if (live)
        walk_hits(n0, p, pinv, chunk_bits, [&](uint32_t o) {
            uint32_t off;
            atomicAdd(&cnt[seg_split(o, seg_bits, seg_log2, rcp, off)], 1u);
        });
    __syncthreads();
    if (t < segs) {
        base[t] = atomicAdd(&bucket_count[seg0 + t], cnt[t]);
        cnt[t] = 0;
    }
    __syncthreads();
    if (live) {
        walk_hits(n0, p, pinv, chunk_bits, [&](uint32_t o) {
            uint32_t off;
            const uint32_t s = seg_split(o, seg_bits, seg_log2, rcp, off);
            const uint32_t slot = base[s] + atomicAdd(&cnt[s], 1u);
            if (slot < depth)
                buckets[static_cast<uint64_t>(seg0 + s) * depth + slot] = off;
            else
                atomicOr(overflow, 1u);
        });
    }
}

__global__ void __launch_bounds__(256) reciprocal_kernel(const uint32_t *primes, uint32_t n, double *inv)
{
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n)
        inv[i] = 1.0 / static_cast<double>(primes[i]);
}

// Static LDS sizes the segment kernels are built for (words of segment).
constexpr uint32_t kSegSizes[] = {512, 2048, 8192, 16384, kWideSegWords};
// (beside the tables and the segment: the item word and the reduction array,
// 132 bytes, with room for alignment)
static_assert(2 * ((kTableWords + kWideSegWords) * 4 + 256) <= 160 * 1024,
              "two workgroups of the widest segment per CU");

}  // namespace

uint32_t seg_capacity_for(uint32_t seg_words)
{
    for (uint32_t c : kSegSizes)
        if (seg_words <= c)
            return c;
    return 0;
}

uint32_t lds_bytes_for(uint32_t seg_words)
{
    const uint32_t cap = seg_capacity_for(seg_words);
    return cap ? (kTableWords + cap) * 4u : 0u;
}

uint32_t max_seg_words()
{
    return kSegSizes[sizeof(kSegSizes) / sizeof(kSegSizes[0]) - 1];
}

hipError_t launch_bootstrap_primes(uint32_t *d_out, uint32_t *d_count, hipStream_t s)
{
    hipLaunchKernelGGL(bootstrap_kernel, dim3(1), dim3(1024), 0, s, d_out, d_count);
    return hipGetLastError();
}

hipError_t launch_bucket_fill(const uint32_t *primes, const double *inv, uint32_t n_large,
                              uint64_t first_odd, uint32_t seg_bits, uint32_t n_segs, uint32_t *buckets,
                              uint32_t *bucket_count, uint32_t depth, uint32_t *overflow, hipStream_t s)
{
    if (n_large == 0 || n_segs == 0)
        return hipSuccess;
    const dim3 grid((n_large + 255) / 256, (n_segs + kBucketChunk - 1) / kBucketChunk);
    hipLaunchKernelGGL(bucket_fill_kernel, grid, dim3(256), 0, s, primes, inv, n_large, first_odd, seg_bits,
                       n_segs, buckets, bucket_count, depth, overflow);
    return hipGetLastError();
}

hipError_t launch_reciprocals(const uint32_t *d_primes, uint32_t n, double *d_inv, hipStream_t s)
{
    if (n == 0)
        return hipSuccess;
    hipLaunchKernelGGL(reciprocal_kernel, dim3((n + 255) / 256), dim3(256), 0, s, d_primes, n, d_inv);
    return hipGetLastError();
}

namespace {
template <uint32_t kSegMax>
void launch_range_cap(const RangeArgs &r, const PrimeArgs &p, uint32_t seg_words, uint32_t threads,
                      uint32_t n_segments, uint32_t chunk, uint32_t n_chunks, uint32_t grid, hipStream_t s)
{
    if (r.out)
        hipLaunchKernelGGL((range_kernel<kSegMax, true>), dim3(grid), dim3(threads), 0, s, r, p, seg_words,
                           n_segments, chunk, n_chunks);
    else
        hipLaunchKernelGGL((range_kernel<kSegMax, false>), dim3(grid), dim3(threads), 0, s, r, p, seg_words,
                           n_segments, chunk, n_chunks);
}

template <uint32_t kSegMax>
void launch_batch_cap(BatchHeader *d_blob, const uint32_t *d_primes, const double *d_inv,
                      uint32_t *d_words, uint32_t *d_item_counts, uint32_t seg_words, uint32_t threads,
                      uint32_t grid, bool small, hipStream_t s)
{
    if (small)
        hipLaunchKernelGGL((batch_kernel<kSegMax, true>), dim3(grid), dim3(threads), 0, s, d_blob, d_primes, d_inv,
                           d_words, d_item_counts, seg_words);
    else
        hipLaunchKernelGGL((batch_kernel<kSegMax, false>), dim3(grid), dim3(threads), 0, s, d_blob, d_primes, d_inv,
                           d_words, d_item_counts, seg_words);
}
}  // namespace

namespace {
template <typename K>
uint32_t occupancy(K kernel, uint32_t threads)
{
    int n = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, kernel, static_cast<int>(threads), 0) != hipSuccess)
        return 1;
    return n > 0 ? static_cast<uint32_t>(n) : 1u;
}

// The occupancy query costs microseconds and its answer depends only on the
// kernel and the workgroup size (every device here is a gfx950), so it is
// asked once per (kernel, threads) and kept; 0 = not asked yet.
std::atomic<uint32_t> g_occupancy[3][6][17];  // [range count, range bitmap, batch]

uint32_t cap_index(uint32_t cap)
{
    switch (cap) {
    case 512: return 1;
    case 2048: return 2;
    case 8192: return 3;
    case 16384: return 4;
    case kWideSegWords: return 5;
    default: return 0;
    }
}

template <typename K>
uint32_t blocks_per_cu(K kernel, uint32_t threads, int kind, uint32_t cap)
{
    const uint32_t ci = cap_index(cap);
    if (threads % 64 != 0 || threads > 1024 || ci == 0)
        return occupancy(kernel, threads);
    std::atomic<uint32_t> &slot = g_occupancy[kind][ci][threads / 64];
    uint32_t v = slot.load(std::memory_order_relaxed);
    if (v == 0) {
        v = occupancy(kernel, threads);
        slot.store(v, std::memory_order_relaxed);
    }
    return v;
}
}  // namespace

uint32_t range_blocks_per_cu(uint32_t seg_words, uint32_t threads, bool write)
{
    const uint32_t cap = seg_capacity_for(seg_words);
    const int kind = write ? 1 : 0;
    switch (cap) {
    case 512: return write ? blocks_per_cu(range_kernel<512, true>, threads, kind, cap) : blocks_per_cu(range_kernel<512, false>, threads, kind, cap);
    case 2048: return write ? blocks_per_cu(range_kernel<2048, true>, threads, kind, cap) : blocks_per_cu(range_kernel<2048, false>, threads, kind, cap);
    case 8192: return write ? blocks_per_cu(range_kernel<8192, true>, threads, kind, cap) : blocks_per_cu(range_kernel<8192, false>, threads, kind, cap);
    case 16384: return write ? blocks_per_cu(range_kernel<16384, true>, threads, kind, cap) : blocks_per_cu(range_kernel<16384, false>, threads, kind, cap);
    case kWideSegWords: return write ? blocks_per_cu(range_kernel<kWideSegWords, true>, threads, kind, cap) : blocks_per_cu(range_kernel<kWideSegWords, false>, threads, kind, cap);
    default: return 1;
    }
}

uint32_t batch_blocks_per_cu(uint32_t seg_words, uint32_t threads)
{
    const uint32_t cap = seg_capacity_for(seg_words);
    switch (cap) {
    case 512: return blocks_per_cu(batch_kernel<512, true>, threads, 2, cap);
    case 2048: return blocks_per_cu(batch_kernel<2048, true>, threads, 2, cap);
    case 8192: return blocks_per_cu(batch_kernel<8192, true>, threads, 2, cap);
    case 16384: return blocks_per_cu(batch_kernel<16384, true>, threads, 2, cap);
    case kWideSegWords: return blocks_per_cu(batch_kernel<kWideSegWords, true>, threads, 2, cap);
    default: return 1;
    }
}

void range_chunks(uint32_t n_segments, uint32_t grid, uint32_t *chunk, uint32_t *n_chunks)
{
    // Beyond two rounds, the last 2 * grid segments go singly; the rest in
    // runs that give each workgroup about three runs.
    if (n_segments > grid && n_segments <= 2 * grid) {
        // Two rounds at most: pairs of consecutive segments, one pair per
        // workgroup, so that the second segment of each pair continues its
        // carried sparse primes and takes the reversed dense order
        // (bitmap of [2, 1e9), 1018 segments on 512 workgroups: 0.0817 ->
        // 0.0735 ms).
        *chunk = 2;
        *n_chunks = n_segments / 2;
        return;
    }
    const uint32_t tail = n_segments < 2 * grid ? n_segments : 2 * grid;
    const uint32_t bulk = n_segments - tail;
    uint32_t c = grid ? bulk / (3 * grid) : 0;
    c = c < kMaxChunk ? c : kMaxChunk;
    if (c < 2) {
        *chunk = 1;
        *n_chunks = 0;
        return;
    }
    *chunk = c;
    *n_chunks = bulk / c;
}

hipError_t launch_range(const RangeArgs &r, const PrimeArgs &p, uint32_t seg_words,
                        uint32_t block_threads, uint32_t n_segments, uint32_t max_blocks, hipStream_t s)
{
    const uint32_t grid = n_segments < max_blocks ? n_segments : max_blocks;
    if (grid == 0)
        return hipSuccess;
    uint32_t chunk = 1, n_chunks = 0;
    range_chunks(n_segments, grid, &chunk, &n_chunks);
    switch (seg_capacity_for(seg_words)) {
    case 512: launch_range_cap<512>(r, p, seg_words, block_threads, n_segments, chunk, n_chunks, grid, s); break;
    case 2048: launch_range_cap<2048>(r, p, seg_words, block_threads, n_segments, chunk, n_chunks, grid, s); break;
    case 8192: launch_range_cap<8192>(r, p, seg_words, block_threads, n_segments, chunk, n_chunks, grid, s); break;
    case 16384: launch_range_cap<16384>(r, p, seg_words, block_threads, n_segments, chunk, n_chunks, grid, s); break;
    case kWideSegWords: launch_range_cap<kWideSegWords>(r, p, seg_words, block_threads, n_segments, chunk, n_chunks, grid, s); break;
    default: return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

uint64_t compact_tmp_words(uint64_t n_words)
{
    return (n_words + kCompactChunk - 1) / kCompactChunk + 1;
}

hipError_t launch_copy_words(const uint32_t *src, uint32_t *dst, uint64_t n_words, hipStream_t s)
{
    if (n_words == 0)
        return hipSuccess;
    // 16 workgroups with four loads in flight per thread already reach the
    // PCIe rate to host memory (measured 52-56 GB/s for 8-64 MiB, as fast as
    // hipMemcpyAsync); more would only hold CU slots (a CU running a
    // sieve launch's two workgroups has none free) that concurrent sieve
    // launches need.
    const uint64_t n16 = (n_words + 3) / 4;
    const uint32_t blocks = static_cast<uint32_t>(n16 < 16 * 256 ? (n16 + 255) / 256 : 16);
    hipLaunchKernelGGL(copy_words_kernel, dim3(blocks), dim3(256), 0, s, reinterpret_cast<const uint4 *>(src),
                       reinterpret_cast<uint4 *>(dst), n_words);
    return hipGetLastError();
}

hipError_t launch_compact(const uint32_t *d_words, uint64_t n_words, uint64_t first_odd,
                          uint32_t *d_tmp, uint32_t *d_out, uint32_t *d_total, hipStream_t s)
{
    const uint32_t nb = static_cast<uint32_t>((n_words + kCompactChunk - 1) / kCompactChunk);
    if (nb == 0)
        return hipMemsetAsync(d_total, 0, sizeof(uint32_t), s);
    hipLaunchKernelGGL(compact_count_kernel, dim3(nb), dim3(kCompactThreads), 0, s, d_words, n_words,
                       d_tmp);
    hipLaunchKernelGGL(compact_scan_kernel, dim3(1), dim3(1024), 0, s, d_tmp, nb, d_total);
    hipLaunchKernelGGL(compact_write_kernel, dim3(nb), dim3(kCompactThreads), 0, s, d_words, n_words,
                       first_odd, d_tmp, d_out);
    return hipGetLastError();
}

hipError_t launch_batch(const void *h_blob, BatchHeader *d_blob, uint32_t max_intervals, const uint32_t *d_primes,
                        const double *d_inv, uint32_t *d_words, uint32_t *d_item_counts,
                        unsigned long long *counts, uint32_t seg_words, uint32_t block_threads,
                        uint32_t n_blocks, bool small, hipStream_t s)
{
    if (n_blocks == 0)
        return hipSuccess;
    hipLaunchKernelGGL(batch_stage_kernel, dim3(kStageBlocks), dim3(256), 0, s, static_cast<const uint4 *>(h_blob),
                       reinterpret_cast<uint4 *>(d_blob));
    switch (seg_capacity_for(seg_words)) {
    case 512: launch_batch_cap<512>(d_blob, d_primes, d_inv, d_words, d_item_counts, seg_words, block_threads, n_blocks, small, s); break;
    case 2048: launch_batch_cap<2048>(d_blob, d_primes, d_inv, d_words, d_item_counts, seg_words, block_threads, n_blocks, small, s); break;
    case 8192: launch_batch_cap<8192>(d_blob, d_primes, d_inv, d_words, d_item_counts, seg_words, block_threads, n_blocks, small, s); break;
    case 16384: launch_batch_cap<16384>(d_blob, d_primes, d_inv, d_words, d_item_counts, seg_words, block_threads, n_blocks, small, s); break;
    case kWideSegWords: launch_batch_cap<kWideSegWords>(d_blob, d_primes, d_inv, d_words, d_item_counts, seg_words, block_threads, n_blocks, small, s); break;
    default: return hipErrorInvalidValue;
    }
    const uint32_t waves_blocks = (max_intervals + 3) / 4;  // four wavefronts per block
    const uint32_t rb = waves_blocks == 0 ? 1 : (waves_blocks < 1024 ? waves_blocks : 1024);
    hipLaunchKernelGGL(batch_reduce_kernel, dim3(rb), dim3(256), 0, s, d_blob, d_item_counts, counts);
    return hipGetLastError();
}

}  // namespace sv
