// The allocation-free variant of the plain range call (declared in sieve.h
// as sieve_range_bitmap_noalloc).
//
// The plain call keeps its work queues and partial counts in a per-context
// counter slot and may grow the base-prime table or the hit-bucket pool on
// demand.  This variant allocates nothing: its counters live in `scratch`, a
// file-scope device array (one per GPU, held until the process ends), the
// base primes must already be resident in the context, and the range is
// sieved without hit buckets (the same result; buckets only change the speed
// beyond about 1.5e12).  The count goes to a caller-owned device word in
// stream order, so the call never waits on the host.
//
// The host never passes `scratch` itself to a kernel: in host code that name
// is a stand-in, not a device address.  At set-up (context creation) the
// device address of each GPU's copy is looked up once with
// hipGetSymbolAddress and kept per device; every later use goes through it.
#include <mutex>

#include "sieve_runtime.h"

namespace {

// One range launch's counter block (work queues, count lines, grid word):
// kCounterWords words, 4,352 bytes.  The range kernel's last workgroup returns
// it to all zero, so it starts every call clean; it is also cleared at
// set-up and after a call that failed once its launch may have been queued.
constexpr uint32_t kScratchWords = sv::kCounterWords;
static __device__ __align__(256) uint32_t scratch[kScratchWords];

constexpr int kMaxDevices = 64;
std::mutex g_mu;
uint32_t *g_scratch[kMaxDevices] = {};  // device address of each GPU's copy
bool g_dirty[kMaxDevices] = {};         // the copy may not be all zero

__global__ void __launch_bounds__(256) scratch_clear_kernel(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x)
        p[i] = 0;
}

__global__ void __launch_bounds__(64) store_count_kernel(unsigned long long *dst, unsigned long long v)
{
    if (threadIdx.x == 0)
        *dst = v;
}

}  // namespace

namespace sv {

int noalloc_setup(sieve_ctx *c)
{
    if (c->device < 0 || c->device >= kMaxDevices)
        return SIEVE_ENODEV;
    std::lock_guard<std::mutex> g(g_mu);
    if (g_scratch[c->device])
        return SIEVE_OK;
    // the context's device is current
    void *ptr = nullptr;
    SV_HIP_TRY(c, hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    if (!ptr)
        return SIEVE_EDEVICE;
    hipLaunchKernelGGL(scratch_clear_kernel, dim3(1), dim3(256), 0, c->stream, static_cast<uint32_t *>(ptr),
                       kScratchWords);
    SV_HIP_TRY(c, hipGetLastError());
    SV_HIP_TRY(c, hipStreamSynchronize(c->stream));
    g_scratch[c->device] = static_cast<uint32_t *>(ptr);
    return SIEVE_OK;
}

}  // namespace sv

extern "C" {

int sieve_range_bitmap_noalloc(sieve_ctx *c, uint64_t lo, uint64_t hi, uint32_t *d_words, uint64_t n_words,
                               unsigned long long *d_pi, void *stream)
{
    if (!c || lo > hi)
        return SIEVE_EINVAL;
    if (hi > SIEVE_MAX_HI)
        return SIEVE_ERANGE;
    if (reinterpret_cast<uintptr_t>(d_words) % 4 != 0 || reinterpret_cast<uintptr_t>(d_pi) % 8 != 0)
        return SIEVE_EINVAL;
    const uint64_t need = sieve_bitmap_words(lo, hi);
    if (d_words && n_words < need)
        return SIEVE_EBUFSZ;
    sieve_tuning t = c->tuning;
    t.bucket_limit = 0xffffffffu;  // no hit buckets: their pool is allocated on demand
    sieve_plan_info pl{};
    if (int st = sv::make_plan(lo, hi, &t, c->n_cu, c->lds_max, &pl))
        return st;
    if (pl.n_segments > 0xffffffffull || pl.sqrt_bound > c->primes_limit)
        return SIEVE_ERANGE;  // the base primes it needs are not resident
    if (c->device < 0 || c->device >= kMaxDevices)
        return SIEVE_ENODEV;
    uint32_t *ctr = nullptr;
    bool dirty = false;
    {
        std::lock_guard<std::mutex> g(g_mu);
        ctr = g_scratch[c->device];
        dirty = g_dirty[c->device];
    }
    if (!ctr)
        return SIEVE_EDEVICE;  // set-up (sieve_create) did not finish
    SV_HIP_TRY(c, hipSetDevice(c->device));
    hipStream_t s = static_cast<hipStream_t>(stream);  // NULL: the default stream
    const uint32_t two = (lo <= 2 && 2 < hi) ? 1u : 0u;
    if (pl.nbits == 0) {
        if (d_pi) {
            hipLaunchKernelGGL(store_count_kernel, dim3(1), dim3(64), 0, s, d_pi,
                               static_cast<unsigned long long>(two));
            SV_HIP_TRY(c, hipGetLastError());
        }
        return SIEVE_OK;
    }
    {
        std::lock_guard<std::mutex> g(g_mu);
        g_dirty[c->device] = true;
    }
    if (dirty) {
        hipLaunchKernelGGL(scratch_clear_kernel, dim3(1), dim3(256), 0, s, ctr, kScratchWords);
        SV_HIP_TRY(c, hipGetLastError());
    }
    uint32_t n_mark = 0, n_dense = 0;
    sv::marking_primes(c, pl.sqrt_bound, pl.dense_limit, &n_mark, &n_dense);
    sv::RangeArgs ra{(lo & ~1ull) + 1, pl.nbits, pl.n_words, d_words, ctr, d_pi != nullptr, true,
                     d_pi, nullptr, nullptr, 0, two};
    sv::PrimeArgs pa{c->d_primes + sv::kPresievePrimes, c->d_inv + sv::kPresievePrimes, n_dense, n_mark};
    SV_HIP_TRY(c, sv::launch_range(ra, pa, pl.seg_bits / 32, pl.block_threads,
                                   static_cast<uint32_t>(pl.n_segments),
                                   sv::resident_blocks(c, pl, d_words != nullptr), s));
    {
        // the launch is queued: it leaves the counters all zero
        std::lock_guard<std::mutex> g(g_mu);
        g_dirty[c->device] = false;
    }
    return SIEVE_OK;
}

}  // extern "C"
