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
//   2. dense primes (37 <= p < dense_limit): one wavefront per prime, lane k
//      marks multiples k, k+64, k+128, ... of the prime's first odd multiple
//      in the segment.  64*p bits is a whole number of words, so each lane's
//      bit position inside a word never changes and its word address grows by
//      2p per mark: one LDS atomic OR and one add per mark;
//   3. sparse primes: one lane per prime walks its few multiples.
// Then every thread counts the unmarked bits of its words (popcount plus a
// wavefront shuffle reduction) and, for bitmap output, stores them to HBM.
//
// Crossing off starts at max(p*p, first odd multiple in the segment), so a
// base prime never marks itself; the pre-sieve does mark 3..31 themselves and
// leaves 1 unmarked, which the first word of a range corrects.
#include "sieve_internal.h"

namespace sv {
namespace {

constexpr uint32_t kLA = 3u * 5u * 7u * 11u * 13u;  // 15015
constexpr uint32_t kLB = 17u * 19u * 23u;           // 7429
constexpr uint32_t kLC = 29u * 31u;                 // 899
// A table of period L holds bits x in [0, L + 63): enough for a 64-bit window
// starting at any phase j < L.
constexpr uint32_t kWA = (kLA - 1) / 32 + 2;  // 471
constexpr uint32_t kWB = (kLB - 1) / 32 + 2;  // 234
constexpr uint32_t kWC = (kLC - 1) / 32 + 2;  // 30
static_assert(kWA + kWB + kWC <= kTableWords, "pre-sieve tables exceed their LDS area");

__device__ __forceinline__ void lds_or(uint32_t *word, uint32_t mask)
{
    __hip_atomic_fetch_or(word, mask, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Bit b of table word k stands for the odd integer 2(32k + b) + 1 and is set
// when one of the group's primes divides it: p | 2x + 1 <=> x = (p-1)/2 mod p.
__device__ void build_table(uint32_t *tab, uint32_t n_words, const uint32_t *ps, int np)
{
    for (uint32_t k = threadIdx.x; k < n_words; k += blockDim.x) {
        uint32_t m = 0;
        for (int i = 0; i < np; ++i) {
            uint32_t p = ps[i];
            uint32_t x0 = 32u * k;
            uint32_t b = ((p - 1) / 2 + p - x0 % p) % p;  // first bit with x = (p-1)/2 mod p
            for (; b < 32; b += p)
                m |= 1u << b;
        }
        tab[k] = m;
    }
}

__device__ void build_tables(uint32_t *tabs)
{
    const uint32_t pa[5] = {3, 5, 7, 11, 13};
    const uint32_t pb[3] = {17, 19, 23};
    const uint32_t pc[2] = {29, 31};
    build_table(tabs, kWA, pa, 5);
    build_table(tabs + kWA, kWB, pb, 3);
    build_table(tabs + kWA + kWB, kWC, pc, 2);
}

// 32 pattern bits starting at phase j of a table: a funnel shift of two
// consecutive table words.
__device__ __forceinline__ uint32_t pattern_at(const uint32_t *tab, uint32_t j)
{
    const uint32_t k = j >> 5;
    return __builtin_amdgcn_alignbit(tab[k + 1], tab[k], j);
}

// n mod p for n < 2^53 and odd p < 2^25, through a double quotient.  n and
// p are exact in double; the rounded quotient is at most one above the true
// floor, which the final correction removes.
__device__ __forceinline__ uint32_t mod_u64(uint64_t n, uint32_t p)
{
    const double q = floor(static_cast<double>(n) / static_cast<double>(p));
    int64_t r = static_cast<int64_t>(n - static_cast<uint64_t>(q) * p);
    if (r < 0)
        r += p;
    else if (r >= static_cast<int64_t>(p))
        r -= p;
    return static_cast<uint32_t>(r);
}

// Bit offset, inside the segment whose bit 0 is the odd integer n0, of the
// first odd multiple m of p with m >= n0 and m >= p*p.  Returns at least
// lim_bits when no such multiple falls before bit lim_bits.
__device__ __forceinline__ uint32_t first_offset(uint64_t n0, uint32_t p, uint32_t lim_bits)
{
    const uint32_t r = mod_u64(n0, p);
    uint32_t d = r ? p - r : 0;  // n0 + d is the first multiple >= n0
    if (d & 1)                   // n0 is odd, so n0 + d is even: take the next one
        d += p;
    const uint64_t p2 = static_cast<uint64_t>(p) * p;
    if (n0 + d < p2) {
        const uint64_t off = (p2 - n0) >> 1;
        return off < lim_bits ? static_cast<uint32_t>(off) : lim_bits;
    }
    return d >> 1;
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

// Sieve segment `seg` of one range into LDS and emit its words and count.
// tabs: the pre-sieve tables in LDS; seg_lds: seg_words_max words of LDS.
template <bool kWrite>
__device__ void sieve_segment(const uint32_t *tabs, uint32_t *seg_lds, uint32_t seg_words_max,
                              uint64_t seg, uint64_t first_odd, uint64_t nbits, uint64_t n_words,
                              const uint32_t *primes, uint32_t n_dense, uint32_t n_primes,
                              uint32_t *out, unsigned long long *count)
{
    const uint32_t t = threadIdx.x;
    const uint32_t nthreads = blockDim.x;
    const uint64_t w0 = seg * seg_words_max;  // first word of the segment in the range
    const uint64_t left = n_words - w0;
    const uint32_t sw = left < seg_words_max ? static_cast<uint32_t>(left) : seg_words_max;
    const uint32_t lim_bits = sw * 32;
    const uint64_t n0 = first_odd + 64 * w0;  // odd integer of the segment's bit 0

    // 1. pre-sieve.  Bit g of the segment is the odd integer 2x + 1 with
    //    x = (n0 >> 1) + g; pattern phases are x mod L.
    {
        const uint64_t x0 = (n0 >> 1) + 32ull * t;
        uint32_t ja = static_cast<uint32_t>(x0 % kLA);
        uint32_t jb = static_cast<uint32_t>(x0 % kLB);
        uint32_t jc = static_cast<uint32_t>(x0 % kLC);
        const uint32_t sa = (32u * nthreads) % kLA;
        const uint32_t sb = (32u * nthreads) % kLB;
        const uint32_t sc = (32u * nthreads) % kLC;
        const uint32_t *ta = tabs;
        const uint32_t *tb = tabs + kWA;
        const uint32_t *tc = tabs + kWA + kWB;
        for (uint32_t w = t; w < sw; w += nthreads) {
            seg_lds[w] = pattern_at(ta, ja) | pattern_at(tb, jb) | pattern_at(tc, jc);
            ja += sa;
            ja = min(ja, ja - kLA);  // unsigned: subtract L once if ja >= L
            jb += sb;
            jb = min(jb, jb - kLB);
            jc += sc;
            jc = min(jc, jc - kLC);
        }
    }
    __syncthreads();

    // 2a. dense primes: one wavefront per prime.  Lane l of wave w computes
    //     the start of prime r*64*nw + l*nw + w, so each wave gets an
    //     interleaved, evenly weighted share of the primes.
    {
        const uint32_t lane = t & 63;
        const uint32_t wave = t >> 6;
        const uint32_t nw = nthreads >> 6;
        for (uint32_t r0 = 0; r0 + wave < n_dense; r0 += 64 * nw) {
            const uint32_t i = r0 + lane * nw + wave;
            uint32_t p = 0, s0 = 0;
            if (i < n_dense) {
                p = primes[i];
                s0 = first_offset(n0, p, lim_bits);
            }
            for (int l = 0; l < 64; ++l) {
                const uint32_t pl = __builtin_amdgcn_readlane(p, l);
                if (pl == 0)
                    break;
                const uint32_t sl = __builtin_amdgcn_readlane(s0, l);
                const uint32_t o = sl + lane * pl;
                const uint32_t mask = 1u << (o & 31);
                const uint32_t step = 2 * pl;  // 64 * p bits = 2p words
                for (uint32_t a = o >> 5; a < sw; a += step)
                    lds_or(seg_lds + a, mask);
            }
        }
    }
    // 2b. sparse primes: one lane per prime.
    for (uint32_t i = n_dense + t; i < n_primes; i += nthreads) {
        const uint32_t p = primes[i];
        for (uint32_t o = first_offset(n0, p, lim_bits); o < lim_bits; o += p)
            lds_or(seg_lds + (o >> 5), 1u << (o & 31));
    }
    __syncthreads();

    // 3. count (and store) the unmarked bits.
    uint32_t c = 0;
    const uint32_t tail = static_cast<uint32_t>(nbits & 31);
    for (uint32_t w = t; w < sw; w += nthreads) {
        uint32_t v = ~seg_lds[w];
        const uint64_t gw = w0 + w;
        if (gw == 0)
            v = fix_first_word(v, first_odd);
        if (tail && gw == n_words - 1)
            v &= (1u << tail) - 1;
        c += __popc(v);
        if (kWrite)
            out[gw] = v;
    }
    c = wave_sum(c);
    if ((t & 63) == 0 && count)
        atomicAdd(count, static_cast<unsigned long long>(c));
    __syncthreads();  // the LDS segment is reused by the next segment
}

template <bool kWrite>
__global__ void __launch_bounds__(1024) range_kernel(RangeArgs r, PrimeArgs pa, uint32_t seg_words,
                                                      uint64_t n_segments)
{
    extern __shared__ uint32_t lds[];
    uint32_t *tabs = lds;
    uint32_t *seg = lds + kTableWords;
    build_tables(tabs);
    __syncthreads();
    for (uint64_t s = blockIdx.x; s < n_segments; s += gridDim.x)
        sieve_segment<kWrite>(tabs, seg, seg_words, s, r.first_odd, r.nbits, r.n_words, pa.primes,
                              pa.n_dense, pa.n_primes, r.out, r.count);
}

// Persistent batch kernel: workgroups pop (interval, segment) items from a
// device counter until the queue is empty.  Every workgroup leaves the loop
// once the counter passes n_items, so the grid always drains.
__global__ void __launch_bounds__(1024) batch_kernel(const BatchInterval *ivs, const uint32_t *item_iv,
                                                      uint32_t n_items, const uint32_t *primes,
                                                      uint32_t *words, unsigned long long *counts,
                                                      uint32_t *queue, uint32_t seg_words)
{
    extern __shared__ uint32_t lds[];
    __shared__ uint32_t item_sh;
    uint32_t *tabs = lds;
    uint32_t *seg = lds + kTableWords;
    build_tables(tabs);
    for (;;) {
        __syncthreads();
        if (threadIdx.x == 0)
            item_sh = atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = item_sh;
        if (item >= n_items)
            break;
        const uint32_t k = item_iv[item];
        const BatchInterval iv = ivs[k];
        const uint64_t s = item - iv.seg_begin;
        if (iv.word_offset != ~0ull)
            sieve_segment<true>(tabs, seg, seg_words, s, iv.first_odd, iv.nbits, iv.n_words, primes,
                                iv.n_dense, iv.n_primes, words + iv.word_offset, counts + k);
        else
            sieve_segment<false>(tabs, seg, seg_words, s, iv.first_odd, iv.nbits, iv.n_words, primes,
                                 iv.n_dense, iv.n_primes, nullptr, counts + k);
    }
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

}  // namespace

uint32_t lds_bytes_for(uint32_t seg_words)
{
    return (kTableWords + seg_words) * 4u;
}

hipError_t launch_bootstrap_primes(uint32_t *d_out, uint32_t *d_count, hipStream_t s)
{
    hipLaunchKernelGGL(bootstrap_kernel, dim3(1), dim3(1024), 0, s, d_out, d_count);
    return hipGetLastError();
}

hipError_t launch_range(const RangeArgs &r, const PrimeArgs &p, uint32_t seg_words,
                        uint32_t block_threads, uint64_t n_segments, hipStream_t s)
{
    const uint32_t lds = lds_bytes_for(seg_words);
    const uint64_t grid = n_segments;  // one workgroup per segment
    if (grid == 0)
        return hipSuccess;
    if (r.out)
        hipLaunchKernelGGL(range_kernel<true>, dim3(static_cast<uint32_t>(grid)), dim3(block_threads),
                           lds, s, r, p, seg_words, n_segments);
    else
        hipLaunchKernelGGL(range_kernel<false>, dim3(static_cast<uint32_t>(grid)), dim3(block_threads),
                           lds, s, r, p, seg_words, n_segments);
    return hipGetLastError();
}

uint64_t compact_tmp_words(uint64_t n_words)
{
    return (n_words + kCompactChunk - 1) / kCompactChunk + 1;
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

hipError_t launch_batch(const BatchInterval *d_iv, uint32_t n_iv, const uint32_t *d_item_iv,
                        uint32_t n_items, const uint32_t *d_primes, uint32_t *d_words,
                        unsigned long long *d_counts, uint32_t *d_queue, uint32_t seg_words,
                        uint32_t block_threads, uint32_t n_blocks, hipStream_t s)
{
    (void)n_iv;
    if (n_items == 0 || n_blocks == 0)
        return hipSuccess;
    hipLaunchKernelGGL(batch_kernel, dim3(n_blocks), dim3(block_threads), lds_bytes_for(seg_words), s,
                       d_iv, d_item_iv, n_items, d_primes, d_words, d_counts, d_queue, seg_words);
    return hipGetLastError();
}

}  // namespace sv
