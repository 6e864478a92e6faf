// Batched primality tests on the GPU: the paper's modular exponentiation by
// repeated squaring (Section 3.2, Alg. 2) driving the Fermat test
// (Alg. 3) and deterministic Miller-Rabin, the test the paper points to for
// Carmichael numbers.  One lane per candidate n < 2^64; products modulo n
// are Montgomery products with R = 2^64 (n odd), so no 128-bit division is
// ever needed.
#include "sieve_runtime.h"

namespace sv {
namespace {

struct Mont {
    uint64_t n;     // odd modulus
    uint64_t ninv;  // -n^-1 mod 2^64
    uint64_t one;   // R mod n
};

// a * b as a 128-bit (lo, hi) pair from 32-bit limbs: four 32 x 32 + 64
// multiply-adds, each partial product formed once.
__device__ __forceinline__ void mul_wide(uint64_t a, uint64_t b, uint64_t &lo, uint64_t &hi)
{
    const uint32_t a0 = static_cast<uint32_t>(a), a1 = static_cast<uint32_t>(a >> 32);
    const uint32_t b0 = static_cast<uint32_t>(b), b1 = static_cast<uint32_t>(b >> 32);
    const uint64_t p00 = static_cast<uint64_t>(a0) * b0;
    const uint64_t t1 = static_cast<uint64_t>(a0) * b1 + (p00 >> 32);
    const uint64_t t2 = static_cast<uint64_t>(a1) * b0 + static_cast<uint32_t>(t1);
    hi = static_cast<uint64_t>(a1) * b1 + (t1 >> 32) + (t2 >> 32);
    lo = (t2 << 32) | static_cast<uint32_t>(p00);
}

// a * b * R^-1 mod n, for a, b < n.
__device__ __forceinline__ uint64_t mont_mul(const Mont &m, uint64_t a, uint64_t b)
{
    uint64_t t_lo, t_hi, qn_lo, qn_hi;
    mul_wide(a, b, t_lo, t_hi);
    const uint64_t q = t_lo * m.ninv;  // t + q*n = 0 mod R
    mul_wide(q, m.n, qn_lo, qn_hi);    // only the high half is used
    // (t + q*n) / R = t_hi + qn_hi + (carry out of t_lo + qn_lo, which is 1
    // exactly when t_lo != 0 since the low halves sum to 0 mod R); it is
    // below 2n, so n comes off once when the sum passed 2^64 or reached n
    unsigned long long c1 = 0, c2 = 0;
    const uint64_t r = __builtin_addcll(t_hi, qn_hi, t_lo != 0 ? 1ull : 0ull, &c1);
    const uint64_t d = __builtin_subcll(r, m.n, 0ull, &c2);
    return (c1 | (c2 ^ 1ull)) ? d : r;
}

__device__ __forceinline__ Mont mont_setup(uint64_t n)
{
    Mont m;
    m.n = n;
    uint64_t inv = n;  // n * n = 1 mod 8 for odd n: 3 correct bits
    for (int i = 0; i < 5; ++i)
        inv *= 2 - n * inv;  // Newton: doubles the correct low bits
    m.ninv = 0 - inv;
    m.one = (0 - n) % n;  // 2^64 mod n
    return m;
}

// x R mod n for x < n: x doubled 64 times modulo n.
__device__ __forceinline__ uint64_t to_mont(const Mont &m, uint64_t x)
{
    for (int i = 0; i < 64; ++i) {
        const bool top = (x >> 63) != 0;
        x <<= 1;
        if (top || x >= m.n)
            x -= m.n;
    }
    return x;
}

// base^e in Montgomery form by right-to-left repeated squaring (Alg. 2: x
// collects the squares y = base^(2^k) for the set bits k of e).
__device__ __forceinline__ uint64_t mont_pow(const Mont &m, uint64_t base_m, uint64_t e)
{
    uint64_t x = m.one;
    uint64_t y = base_m;
    while (e) {
        if (e & 1)
            x = mont_mul(m, x, y);
        e >>= 1;
        if (e)
            y = mont_mul(m, y, y);
    }
    return x;
}

// x + y mod n for x, y < n (the sum may pass 2^64).
__device__ __forceinline__ uint64_t add_mod(uint64_t x, uint64_t y, uint64_t n)
{
    const uint64_t s = x + y;
    return (s < x || s >= n) ? s - n : s;
}

// 2^e in Montgomery form (2^e R mod n), e >= 1, by left-to-right repeated
// squaring: the same squarings as mont_pow, but a set bit of e multiplies by
// the base 2, which is one modular doubling instead of a product.
__device__ __forceinline__ uint64_t mont_pow2(const Mont &m, uint64_t e)
{
    int k = 63 - __clzll(e);              // the top bit of e ...
    uint64_t x = add_mod(m.one, m.one, m.n);  // ... is the base itself: 2R mod n
    while (k-- > 0) {
        x = mont_mul(m, x, x);
        if ((e >> k) & 1)
            x = add_mod(x, x, m.n);
    }
    return x;
}

// The end of a Miller-Rabin round from x = a^d R mod n (n - 1 = d * 2^s, d
// odd): true when the base does not prove n composite.
__device__ __forceinline__ bool mr_finish(const Mont &m, uint64_t x, int s)
{
    const uint64_t minus_one = m.n - m.one;  // (n - 1) R mod n
    if (x == m.one || x == minus_one)
        return true;
    for (int j = 1; j < s; ++j) {
        x = mont_mul(m, x, x);
        if (x == minus_one)
            return true;
    }
    return false;
}

// a^e in Montgomery form by left-to-right repeated squaring over fixed
// two-bit windows of e: each window squares twice and multiplies once by
// 1, a, a^2 or a^3 (the product by 1 = R mod n leaves x as it is).  Every
// lane runs the same 32 windows, so a wavefront of different exponents
// never diverges; the right-to-left loop of mont_pow multiplies only on set
// bits, but across 64 lanes some lane almost always has one, so a wavefront
// pays the product on nearly every bit.
__device__ __forceinline__ uint64_t mont_pow_w2(const Mont &m, uint64_t a_m, uint64_t e)
{
    const uint64_t a2 = mont_mul(m, a_m, a_m);
    const uint64_t a3 = mont_mul(m, a2, a_m);
    uint64_t x = m.one;
    for (int k = 62; k >= 0; k -= 2) {
        x = mont_mul(m, x, x);
        x = mont_mul(m, x, x);
        const uint32_t w = static_cast<uint32_t>(e >> k) & 3u;
        const uint64_t t = (w & 2) ? ((w & 1) ? a3 : a2) : ((w & 1) ? a_m : m.one);
        x = mont_mul(m, x, t);
    }
    return x;
}

// One Miller-Rabin round on a base already in Montgomery form (a R mod n,
// a not divisible by n).
__device__ __forceinline__ bool mr_round(const Mont &m, uint64_t a_m, uint64_t d, int s)
{
    return mr_finish(m, mont_pow_w2(m, a_m, d), s);
}

// Deterministic Miller-Rabin for n < 2^64, in three stages so that the
// expensive rounds run on densely packed lanes (see mr_kernel).  Below
// 341550071728321 the bases are the first k primes, k from the published
// bounds below which those bases admit no strong pseudoprime (Jaeschke
// 1993); above it, the seven bases 2, 325, 9375, 28178, 450775, 9780504,
// 1795265022, which admit none below 2^64 (Sinclair 2011, checked against
// the Feitsma-Galway list of base-2 pseudoprimes).
constexpr uint32_t kSmallBases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
constexpr uint64_t kWideBases[7] = {2, 325, 9375, 28178, 450775, 9780504, 1795265022};

// Rounds needed for n >= 41^2 (the first k small bases, or the 7 wide ones).
__device__ __forceinline__ int mr_rounds(uint64_t n, bool &wide)
{
    wide = false;
    if (n < 2047ull)
        return 1;
    if (n < 1373653ull)
        return 2;
    if (n < 25326001ull)
        return 3;
    if (n < 3215031751ull)
        return 4;
    if (n < 2152302898747ull)
        return 5;
    if (n < 3474749660383ull)
        return 6;
    if (n < 341550071728321ull)
        return 7;
    wide = true;
    return 7;
}

// Divisibility by an odd constant p without a division (Granlund and
// Montgomery, 1994): multiplying by p^-1 mod 2^64 maps the multiples of p
// onto [0, (2^64 - 1) / p] and every other n above it.
struct DivTest {
    uint64_t inv;  // p^-1 mod 2^64
    uint64_t lim;  // (2^64 - 1) / p
};

constexpr uint64_t inverse_mod_2_64(uint64_t p)
{
    uint64_t inv = p;  // correct to 3 bits for odd p
    for (int i = 0; i < 5; ++i)
        inv *= 2 - p * inv;
    return inv;
}

struct DivTests {
    DivTest t[12];
};

constexpr DivTests make_div_tests()
{
    DivTests d{};
    for (int i = 1; i < 12; ++i)  // the odd small bases 3..37
        d.t[i] = DivTest{inverse_mod_2_64(kSmallBases[i]), ~0ull / kSmallBases[i]};
    return d;
}

constexpr DivTests kDivTests = make_div_tests();
static_assert(3ull * kDivTests.t[1].inv == 1 && 37ull * kDivTests.t[11].inv == 1, "inverses mod 2^64");

// Stage 1: 0 = composite, 1 = prime, 2 = undecided (no factor up to 37,
// n >= 41^2).
__device__ __forceinline__ uint32_t mr_stage1(uint64_t n)
{
    if (n < 2)
        return 0;
    if ((n & 1) == 0)
        return n == 2 ? 1 : 0;
#pragma unroll
    for (int i = 1; i < 12; ++i) {
        if (n == kSmallBases[i])
            return 1;
        if (n * kDivTests.t[i].inv <= kDivTests.t[i].lim)
            return 0;
    }
    return n < 41 * 41 ? 1 : 2;  // no factor up to 37 and below 41^2: prime
}

__device__ __forceinline__ void mr_split(uint64_t n, uint64_t &d, int &s)
{
    d = n - 1;
    s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        ++s;
    }
}

// Stage 2, for an undecided n: the base-2 round, which rejects almost every
// composite (2^d by squaring and doubling, see mont_pow2).  0 = composite,
// 1 = prime (base 2 is all n < 2047 needs), 2 = undecided.
__device__ __forceinline__ uint32_t mr_stage2(uint64_t n)
{
    uint64_t d;
    int s;
    mr_split(n, d, s);
    const Mont m = mont_setup(n);
    if (!mr_finish(m, mont_pow2(m, d), s))
        return 0;
    bool wide;
    return mr_rounds(n, wide) == 1 ? 1 : 2;
}

// Stage 3: the remaining bases.  Every base is below n here (n >= 41^2 for
// the small bases, n > 3.4e14 for the wide ones), so none is a multiple of
// n; each enters Montgomery form through one product with R^2 mod n.
__device__ __forceinline__ uint32_t mr_stage3(uint64_t n)
{
    uint64_t d;
    int s;
    mr_split(n, d, s);
    const Mont m = mont_setup(n);
    bool wide;
    const int rounds = mr_rounds(n, wide);
    const uint64_t r2 = to_mont(m, m.one);  // R^2 mod n
    for (int i = 1; i < rounds; ++i) {
        const uint64_t a = wide ? kWideBases[i] : kSmallBases[i];
        if (!mr_round(m, mont_mul(m, a, r2), d, s))
            return 0;
    }
    return 1;
}

// One workgroup takes chunks of kMrChunk candidates: every lane runs stage 1
// on its share and queues the undecided ones in LDS; the queue is then
// worked off densely by stage 2, whose survivors (mostly primes) form a
// second queue for stage 3.  Without the queues nearly every wave would
// carry a prime through all its rounds with most lanes idle.
constexpr uint32_t kMrThreads = 256;
constexpr uint32_t kMrChunk = 4096;

__global__ void __launch_bounds__(kMrThreads) mr_kernel(const uint64_t *ns, uint64_t count, uint8_t *out)
{
    __shared__ uint32_t q1[kMrChunk], q2[kMrChunk];
    __shared__ uint32_t n1, n2;
    const uint32_t t = threadIdx.x;
    for (uint64_t base = static_cast<uint64_t>(blockIdx.x) * kMrChunk; base < count;
         base += static_cast<uint64_t>(gridDim.x) * kMrChunk) {
        if (t == 0) {
            n1 = 0;
            n2 = 0;
        }
        __syncthreads();
        const uint32_t here = static_cast<uint32_t>(count - base < kMrChunk ? count - base : kMrChunk);
        for (uint32_t j = t; j < here; j += kMrThreads) {
            const uint32_t v = mr_stage1(ns[base + j]);
            if (v == 2)
                q1[atomicAdd(&n1, 1u)] = j;
            else
                out[base + j] = static_cast<uint8_t>(v);
        }
        __syncthreads();
        for (uint32_t e = t; e < n1; e += kMrThreads) {
            const uint32_t j = q1[e];
            const uint32_t v = mr_stage2(ns[base + j]);
            if (v == 2)
                q2[atomicAdd(&n2, 1u)] = j;
            else
                out[base + j] = static_cast<uint8_t>(v);
        }
        __syncthreads();
        for (uint32_t e = t; e < n2; e += kMrThreads) {
            const uint32_t j = q2[e];
            out[base + j] = static_cast<uint8_t>(mr_stage3(ns[base + j]));
        }
        __syncthreads();  // the queues are reused by the next chunk
    }
}

// a * b mod n for any n > 1 by doubling and adding (64 steps).
__device__ uint64_t mul_mod_slow(uint64_t a, uint64_t b, uint64_t n)
{
    uint64_t r = 0;
    a %= n;
    while (b) {
        if (b & 1)
            r = add_mod(r, a, n);
        a = add_mod(a, a, n);
        b >>= 1;
    }
    return r;
}

// Alg. 3: n passes when a^(n-1) = 1 mod n for every base a_j =
// draws[j] mod (n - 1) + 1; n = 1 (and 0) fail, n = 2 passes.
__global__ void __launch_bounds__(256) fermat_kernel(const uint64_t *ns, uint64_t count, const uint64_t *draws,
                                                     uint32_t iterations, uint8_t *out)
{
    for (uint64_t i = blockIdx.x * uint64_t(blockDim.x) + threadIdx.x; i < count;
         i += uint64_t(gridDim.x) * blockDim.x) {
        const uint64_t n = ns[i];
        uint8_t pass = 1;
        if (n <= 1) {
            pass = 0;
        } else if (n == 2) {
            pass = 1;
        } else if ((n & 1) == 0) {
            // even n > 2 has no Montgomery form: shift-and-add products
            for (uint32_t j = 0; j < iterations && pass; ++j) {
                const uint64_t a = draws[j] % (n - 1) + 1;
                uint64_t x = 1, y = a, e = n - 1;
                while (e) {
                    if (e & 1)
                        x = mul_mod_slow(x, y, n);
                    y = mul_mod_slow(y, y, n);
                    e >>= 1;
                }
                pass = x == 1 ? 1 : 0;
            }
        } else {
            const Mont m = mont_setup(n);
            const uint64_t r2 = to_mont(m, m.one);  // R^2 mod n
            for (uint32_t j = 0; j < iterations && pass; ++j) {
                const uint64_t a = draws[j] % (n - 1) + 1;  // a < n
                pass = mont_pow(m, mont_mul(m, a, r2), n - 1) == m.one ? 1 : 0;
            }
        }
        out[i] = pass;
    }
}

}  // namespace

hipError_t launch_is_prime(const uint64_t *d_n, uint64_t count, uint8_t *d_out, uint32_t blocks, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(mr_kernel, dim3(blocks), dim3(kMrThreads), 0, s, d_n, count, d_out);
    return hipGetLastError();
}

hipError_t launch_fermat(const uint64_t *d_n, uint64_t count, const uint64_t *d_draws, uint32_t iterations,
                         uint8_t *d_out, uint32_t blocks, hipStream_t s)
{
    if (count == 0)
        return hipSuccess;
    hipLaunchKernelGGL(fermat_kernel, dim3(blocks), dim3(256), 0, s, d_n, count, d_draws, iterations, d_out);
    return hipGetLastError();
}

}  // namespace sv

extern "C" {

int sieve_is_prime_batch(sieve_ctx *c, const uint64_t *d_n, uint64_t count, uint8_t *d_out, void *stream)
{
    if (!c || (count && (!d_n || !d_out)))
        return SIEVE_EINVAL;
    if (count == 0)
        return SIEVE_OK;
    SV_HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    const uint64_t want = (count + sv::kMrChunk - 1) / sv::kMrChunk;  // one chunk per workgroup pass
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>(want, 16ull * c->n_cu));
    c->ev_valid = false;
    if (c->timing)
        SV_HIP_TRY(c, hipEventRecord(c->ev_start, s));
    SV_HIP_TRY(c, sv::launch_is_prime(d_n, count, d_out, blocks, s));
    if (c->timing) {
        SV_HIP_TRY(c, hipEventRecord(c->ev_stop, s));
        c->ev_valid = true;
    }
    return SIEVE_OK;
}

int sieve_fermat_batch(sieve_ctx *c, const uint64_t *d_n, uint64_t count, const uint64_t *d_draws,
                       uint32_t iterations, uint8_t *d_out, void *stream)
{
    if (!c || (count && (!d_n || !d_out)) || (iterations && !d_draws))
        return SIEVE_EINVAL;
    if (count == 0)
        return SIEVE_OK;
    SV_HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    const uint64_t want = (count + 255) / 256;
    const uint32_t blocks = static_cast<uint32_t>(std::min<uint64_t>(want, 64ull * c->n_cu));
    c->ev_valid = false;
    if (c->timing)
        SV_HIP_TRY(c, hipEventRecord(c->ev_start, s));
    SV_HIP_TRY(c, sv::launch_fermat(d_n, count, d_draws, iterations, d_out, blocks, s));
    if (c->timing) {
        SV_HIP_TRY(c, hipEventRecord(c->ev_stop, s));
        c->ev_valid = true;
    }
    return SIEVE_OK;
}

}  // extern "C"
