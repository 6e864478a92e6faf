/*
 * sieve.h - C ABI of the MI355X (gfx950) exact range sieve of Eratosthenes.
 *
 * The library finds the primes in a half-open integer range [lo, hi) and
 * counts them.  This is the problem the paper states: the sieve of
 * Eratosthenes finds every prime up to a limit by crossing off the multiples
 * of each prime (Section 1; Section 3.1), and pi(x) counts the primes up to x
 * (Section 1).  The paper splits n integers into ceil(n/k) blocks that
 * workers sieve independently (Section 3.1, Eq. 3); here the blocks are
 * LDS-sized segments that GPU workgroups sieve independently.
 *
 * Conventions shared by every call
 * --------------------------------
 * Status: every call returns a sieve_status (0 = success, negative = error)
 *   and never throws.  On error the outputs are left untouched, except
 *   *n_out on SIEVE_EBUFSZ (set to the size needed).  Arguments are checked
 *   before any device work starts.
 * Domain: 0 <= lo <= hi <= SIEVE_MAX_HI.  lo == hi is valid (an empty range:
 *   pi = 0, zero bitmap words).
 * Bitmap layout: bit i stands for the odd integer (lo & ~1) + 2*i + 1, for
 *   0 <= i < hi/2 - lo/2 (integer division).  Bits are packed least
 *   significant first into little-endian uint32 words: bit i is bit (i % 32)
 *   of word i / 32.  1 means prime.  Bits past the end of the range in the
 *   last word are 0.  The even prime 2 has no bit but is counted in pi when
 *   lo <= 2 < hi.
 * Device buffers: pointers named d_* are device (HBM) addresses on the
 *   context's device, for example the data_ptr() of a torch tensor.  The
 *   caller owns them; the library never frees them.
 * Streams: a `stream` argument is a hipStream_t on the context's device;
 *   NULL is the device's default (null) stream, as in HIP.  Work is ordered on
 *   that stream.
 * Threads: a context is used by one host thread at a time.
 */
#ifndef SIEVE_H
#define SIEVE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#ifndef SIEVE_API
#define SIEVE_API __attribute__((visibility("default")))
#endif

typedef enum sieve_status {
    SIEVE_OK = 0,
    SIEVE_EINVAL = -1,    /* NULL where a pointer is required, lo > hi, bad tuning */
    SIEVE_ERANGE = -2,    /* hi > SIEVE_MAX_HI */
    SIEVE_ENOMEM = -3,    /* device or host allocation failed, or over the HBM budget */
    SIEVE_EBUFSZ = -4,    /* output buffer too small; *n_out holds the size needed */
    SIEVE_EDEVICE = -5,   /* a HIP call failed; see sieve_last_hip_error() */
    SIEVE_ENODEV = -6,    /* no usable gfx950 device */
    SIEVE_EOVERFLOW = -7  /* a bucket pool overflowed and the retry failed */
} sieve_status;

/* Largest accepted hi: 10^15.  sqrt(10^15) < 2^25, so base primes fit in 25
 * bits and every product the kernels form fits in 64 bits. */
#define SIEVE_MAX_HI 1000000000000000ULL

/* Opaque context: owns the device-resident base-prime table, per-call
 * counters, batch work queues and the context stream. */
typedef struct sieve_ctx sieve_ctx;

/* Tuning knobs.  A zero field means "choose automatically".
 *   seg_bits      odd integers per LDS segment (a multiple of 4096, at most
 *                 622,592 = 19,456 words, the most that two workgroups per
 *                 CU can each hold).  Automatic: a power of two giving about
 *                 two segments per workgroup slot, at most 2^19.  A range of
 *                 at least four rounds of 2^19-bit segments (8 per CU) takes
 *                 622,592, and one of two to four rounds without hit buckets
 *                 takes the smallest multiple of 4096 that still needs only
 *                 that many rounds (every round full).
 *   dense_limit   base primes below this are marked by a whole wavefront per
 *                 prime (each lane on four residue classes of the multiples);
 *                 primes at or above it by one lane per prime.  Clamped to
 *                 >= 37; automatic: max(seg_bits / 512, 128).
 *   bucket_limit  base primes at or above this (and at least seg_bits) are
 *                 not scanned per segment: a fill kernel first sorts their
 *                 hits into per-segment buckets in HBM, which the segment
 *                 kernel then applies (plain path, any seg_bits).
 *                 0 = automatic (buckets when sqrt(hi) >= 2 *
 *                 seg_bits and the range holds at least 2^30 odd integers),
 *                 0xFFFFFFFF = never.
 *   bucket_depth  entries per segment bucket (0 = from the expected hits
 *                 plus six standard deviations).  A bucket that overflows is
 *                 detected and the call is redone with twice the depth, so
 *                 results never depend on it.
 *   block_threads threads per workgroup: 256, 512 or 1024 (automatic: 1024
 *                 above 2^18-bit segments, 512 from 2^14, else 256).
 *   wg_per_cu     resident workgroups per compute unit for persistent
 *                 launches (0 = as many as LDS allows). */
typedef struct sieve_tuning {
    uint32_t seg_bits;
    uint32_t dense_limit;
    uint32_t bucket_limit;
    uint32_t bucket_depth;
    uint32_t block_threads;
    uint32_t wg_per_cu;
} sieve_tuning;

/* What a call on [lo, hi) will do, from sieve_plan (pure host arithmetic). */
typedef struct sieve_plan_info {
    uint64_t nbits;        /* odd integers in [lo, hi) = bitmap bits */
    uint64_t n_words;      /* uint32 words of the bitmap */
    uint64_t sqrt_bound;   /* isqrt(hi - 1): largest possible base prime */
    uint64_t n_segments;   /* LDS segments the range is cut into */
    uint32_t seg_bits;     /* odd integers per segment (tuning resolved) */
    uint32_t dense_limit;  /* resolved */
    uint32_t block_threads;/* resolved */
    uint32_t bucket_limit; /* resolved: primes >= this use hit buckets, 0 = none */
} sieve_plan_info;

/* Create a context on HIP device `hip_device`.  hbm_budget_bytes caps the
 * device memory the batch and serving paths may hold at once (0 = 32 GiB).
 * Builds the base-prime table on the device (primes <= 2^20) before
 * returning.  Errors: SIEVE_EINVAL (ctx NULL), SIEVE_ENODEV (no such device,
 * or not gfx950), SIEVE_ENOMEM, SIEVE_EDEVICE.  On success *ctx must be
 * released with sieve_destroy. */
SIEVE_API int sieve_create(sieve_ctx **ctx, int hip_device, uint64_t hbm_budget_bytes);

/* Release a context and everything it owns.  Waits for its stream and for
 * its asynchronous calls still running on other streams.  NULL is accepted
 * and ignored. */
SIEVE_API int sieve_destroy(sieve_ctx *ctx);

/* Static English text for a status code (never NULL). */
SIEVE_API const char *sieve_strerror(int status);

/* The hipError_t of the last failed HIP call on this context (0 if none). */
SIEVE_API int sieve_last_hip_error(const sieve_ctx *ctx);

/* Kernel timing on (on != 0) or off (the default).  While it is on, every
 * sieve call records a HIP event on its stream immediately before and after
 * its kernel launch (or batch graph), for sieve_last_kernel_ms; the two
 * records add a few microseconds to each call, which is why they are off
 * unless asked for.  Turning it off forgets the last timing.  Errors:
 * SIEVE_EINVAL (NULL ctx). */
SIEVE_API int sieve_set_timing(sieve_ctx *ctx, int on);

/* Device time in milliseconds of the last sieve kernel this context launched
 * while timing was on (sieve_range_count, sieve_range_bitmap, sieve_batch,
 * sieve_is_prime_batch or sieve_fermat_batch), from the HIP events recorded
 * around the launch.  Waits for that kernel.  Errors: SIEVE_EINVAL (NULL
 * arguments, timing off, or no timed launch since it was turned on),
 * SIEVE_EDEVICE. */
SIEVE_API int sieve_last_kernel_ms(sieve_ctx *ctx, double *ms);

/* Read or replace the context's tuning.  set validates every field first
 * (SIEVE_EINVAL leaves the old tuning in place). */
SIEVE_API int sieve_get_tuning(const sieve_ctx *ctx, sieve_tuning *out);
SIEVE_API int sieve_set_tuning(sieve_ctx *ctx, const sieve_tuning *tuning);

/* Plan a call on [lo, hi) with the given tuning (NULL = all automatic) for
 * a device with n_cu compute units and lds_bytes of LDS per workgroup.  Pure
 * host arithmetic, no device needed.  Errors as for sieve_range_count. */
SIEVE_API int sieve_plan(uint64_t lo, uint64_t hi, const sieve_tuning *tuning, uint32_t n_cu,
               uint32_t lds_bytes, sieve_plan_info *out);

/* Number of uint32 words of the bitmap of [lo, hi):
 * ceil((hi/2 - lo/2) / 32).  Pure; 0 when lo >= hi. */
SIEVE_API uint64_t sieve_bitmap_words(uint64_t lo, uint64_t hi);

/* The base primes: all primes p <= limit in ascending order, including 2.
 * The paper's sieve crosses off the multiples of every prime up to the
 * square root of the limit (Section 1, where trial division also stops at
 * sqrt(n); Section 3.1), so a range [lo, hi) needs the primes up to
 * isqrt(hi - 1).  They are copied into the HOST buffer out[0 .. cap).  The
 * table is computed on the device (a one-workgroup bootstrap sieve below
 * 2^16, then the range sieve and a compaction kernel) and kept resident in
 * the context.
 * limit <= isqrt(SIEVE_MAX_HI) + 1.  out == NULL or cap == 0 is a size query:
 * only *n_out is written.  Errors: SIEVE_EINVAL (ctx or n_out NULL),
 * SIEVE_ERANGE (limit too large), SIEVE_EBUFSZ (cap < count; *n_out = count),
 * SIEVE_ENOMEM, SIEVE_EDEVICE. */
SIEVE_API int sieve_base_primes(sieve_ctx *ctx, uint64_t limit, uint32_t *out, uint64_t cap,
                      uint64_t *n_out);

/* pi over [lo, hi): the number of primes p with lo <= p < hi, i.e.
 * pi(hi - 1) - pi(lo - 1) for the prime-counting function pi(x) of Section 1.
 * The range is sieved as the paper's Section 3.1 describes (the multiples of
 * each base prime crossed off, the n integers cut into ceil(n/k) blocks
 * that are sieved independently, Eq. 3), each block an LDS segment.  No
 * bitmap is written.  Blocks until *pi_out is valid: it returns as soon as
 * the launch's last workgroup has published the count to pinned host
 * memory, without synchronising `stream` (later work on the
 * stream stays ordered after the launch).
 * Errors: SIEVE_EINVAL (ctx or pi_out NULL, lo > hi), SIEVE_ERANGE,
 * SIEVE_ENOMEM, SIEVE_EDEVICE. */
SIEVE_API int sieve_range_count(sieve_ctx *ctx, uint64_t lo, uint64_t hi, uint64_t *pi_out,
                      void *stream);

/* The primes of [lo, hi) themselves (the sieve of Section 1 lists every
 * prime up to its limit), sieved block by block as in Section 3.1 (Eq. 3),
 * as an odd-only bitmap written to the DEVICE
 * buffer d_words[0 .. n_words); words past sieve_bitmap_words(lo, hi) are not
 * touched.  d_words must be 4-byte aligned.  The words are written in
 * stream order: later work on `stream` (a copy, a kernel, torch operations on
 * that stream) sees them; synchronise `stream` before reading them any other
 * way.  With pi_out == NULL the call returns at once; otherwise it returns
 * as soon as the launch's last workgroup has published pi to pinned host
 * memory (without synchronising `stream`) and stores it.
 * Errors: SIEVE_EINVAL (ctx NULL, d_words NULL with a non-empty range,
 * misaligned d_words, lo > hi), SIEVE_ERANGE, SIEVE_EBUFSZ (n_words too
 * small), SIEVE_ENOMEM, SIEVE_EDEVICE. */
SIEVE_API int sieve_range_bitmap(sieve_ctx *ctx, uint64_t lo, uint64_t hi, uint32_t *d_words,
                       uint64_t n_words, uint64_t *pi_out, void *stream);

/* For callers that cannot allocate device memory: code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc.  The same
 * sieve as sieve_range_bitmap (and, with d_words == NULL, as
 * sieve_range_count), computing exactly the same words and count, but the
 * call allocates nothing (no hipMalloc, hipFree or allocating library
 * routine) and never waits on the host:
 *   - the launch's work queues and partial counts live in a 4,352-byte
 *     device array inside the library, one per GPU, held until the process
 *     ends (its address is looked up by sieve_create);
 *   - the base primes must already be resident in ctx: isqrt(hi - 1) must
 *     not exceed the context's table (2^20 after sieve_create, i.e. any
 *     hi <= 1,099,513,724,929; grow it beforehand with sieve_base_primes);
 *   - no hit buckets are used (their pool is allocated on demand), so
 *     ranges above about 1.5e12 run slower than through sieve_range_bitmap,
 *     with the same result.
 * d_words: DEVICE buffer of n_words >= sieve_bitmap_words(lo, hi) words, or
 *   NULL to count only.  d_pi: DEVICE word (8-byte aligned) that receives
 *   pi over [lo, hi) (the even prime 2 included), or NULL.  Both are written
 *   in stream order on `stream` (NULL = default stream); the call returns
 *   once the work is queued.
 * Every call on one GPU shares that GPU's counter array: calls that overlap
 * on one GPU (from several host threads, or on several streams without an
 * order between them) race and give wrong counts.  Order them on one stream.
 * Errors: SIEVE_EINVAL (ctx NULL, lo > hi, misaligned pointers),
 * SIEVE_ERANGE (hi > SIEVE_MAX_HI, or base primes beyond the resident
 * table), SIEVE_EBUFSZ (n_words too small), SIEVE_ENODEV, SIEVE_EDEVICE. */
SIEVE_API int sieve_range_bitmap_noalloc(sieve_ctx *ctx, uint64_t lo, uint64_t hi, uint32_t *d_words,
                                         uint64_t n_words, unsigned long long *d_pi, void *stream);

/* One interval of a batch.  flags bit 0: write its bitmap at
 * d_words[word_offset ..); the range's words must lie inside total_words. */
typedef struct sieve_interval {
    uint64_t lo;
    uint64_t hi;
    uint64_t word_offset;
    uint32_t flags;
    uint32_t pad;
} sieve_interval;

#define SIEVE_WANT_BITMAP 1u

/* Many independent intervals in one persistent launch (the block partition
 * of Section 3.1, Eq. 3, generalised to many ranges of uneven position and
 * length): every (interval, segment) pair is one work item of a device work
 * queue that resident workgroups drain.  iv is a HOST array of n intervals;
 * pi_out is a HOST array of n counts (pi of each interval).  d_words may be
 * NULL when no interval sets SIEVE_WANT_BITMAP.  Blocks until pi_out is
 * valid.  Intervals may overlap in value; their bitmap word ranges must not
 * overlap.  Errors: SIEVE_EINVAL (NULL pointers, lo > hi in any interval,
 * overlapping or misaligned outputs), SIEVE_ERANGE, SIEVE_EBUFSZ (an
 * interval's words exceed total_words), SIEVE_ENOMEM (work exceeds the HBM
 * budget), SIEVE_EDEVICE. */
SIEVE_API int sieve_batch(sieve_ctx *ctx, const sieve_interval *iv, uint32_t n, uint32_t *d_words,
                uint64_t total_words, uint64_t *pi_out, void *stream);

/* Batched primality of 64-bit integers (the paper's Section 3.2): out[i] = 1
 * when n[i] is prime.  Deterministic Miller-Rabin (the test the paper points
 * to): below 341,550,071,728,321 the bases are the first k <= 7 primes, from
 * the published bounds below which they admit no strong pseudoprime; above
 * it the seven bases 2, 325, 9375, 28178, 450775, 9780504, 1795265022, which
 * admit none below 2^64.  The modular powers are repeated squaring (Alg. 2)
 * in Montgomery form, taken from the top bit down.  d_n and d_out are DEVICE
 * arrays of count entries (uint64, uint8).  Asynchronous on `stream`;
 * sieve_last_kernel_ms times it (timing on).  Errors: SIEVE_EINVAL (NULL
 * arrays), SIEVE_EDEVICE. */
SIEVE_API int sieve_is_prime_batch(sieve_ctx *ctx, const uint64_t *d_n, uint64_t count, uint8_t *d_out,
                                   void *stream);

/* The paper's Fermat test (Alg. 3) on a batch: out[i] = 1 when
 * a^(n-1) = 1 (mod n) for every base a_j = d_draws[j] mod (n - 1) + 1,
 * j < iterations (the caller supplies the random draws; DEVICE array).  n = 0
 * and 1 fail, n = 2 passes.  Carmichael numbers pass for bases prime to them,
 * as the paper warns.  Arguments and errors as for sieve_is_prime_batch. */
SIEVE_API int sieve_fermat_batch(sieve_ctx *ctx, const uint64_t *d_n, uint64_t count, const uint64_t *d_draws,
                                 uint32_t iterations, uint8_t *d_out, void *stream);

/* Autotuner.  Times candidate tunings on the given work and returns the
 * fastest in *best (and its kernel time in *best_ms if not NULL).  The
 * candidates are the automatic plan first (so the answer is never slower
 * than the untuned context), then four segment sizes, each with a matching
 * workgroup size and three dense/sparse bounds.  The winner is then refined:
 * one or two resident workgroups per CU, and, for a single range that uses
 * hit buckets, a large-prime threshold of 2x or 4x the segment size, or no
 * buckets.  One interval is timed as sieve_range_count, several as a
 * sieve_batch in which the intervals that set SIEVE_WANT_BITMAP write their
 * bitmaps (at their word_offset, into a scratch device buffer the tuner
 * allocates for the batch's extent and frees before returning).  Results are cached per context by (single range
 * or batch, decade of the largest hi, log2 of the total bitmap words); a
 * cached answer is returned without timing unless SIEVE_TUNE_FORCE is set.
 * With SIEVE_TUNE_APPLY the context keeps the winner; otherwise its tuning
 * is left as it was.  The candidate search is the project's own (it is not
 * in the paper).  Errors as for sieve_range_count / sieve_batch. */
#define SIEVE_TUNE_APPLY 1u
#define SIEVE_TUNE_FORCE 2u
SIEVE_API int sieve_autotune(sieve_ctx *ctx, const sieve_interval *iv, uint32_t n, uint32_t flags,
                             sieve_tuning *best, double *best_ms);

/* Measured peaks of the two units the sieve kernels load, on this device.
 * The crossing-off of the paper's sieve (Section 3.1) is one 32-bit LDS
 * atomic OR per marked multiple, and the segment kernels' address and
 * start arithmetic runs on the int32 vector ALU (VALU), so the speed of
 * light of a launch is set by these two rates (the paper frames speedup
 * against such limits in Section 2.2, Eq. 1-2).  Each rate comes from a
 * small bounded kernel on every CU (two 1024-thread workgroups per CU, as
 * the sieve kernels run), timed with HIP events after one warm-up launch.
 * The shader clock during a kernel is measured from its own cycle and wall
 * counters. */
typedef struct sieve_peaks {
    double lds_or_lane_ops_per_s;         /* ds_or_b32, each half-wavefront on 32 distinct banks */
    double lds_or_lanes_per_clk_cu;       /* the same per CU per shader clock */
    double lds_write_lane_ops_per_s;      /* ds_write_b32, same addresses */
    double lds_or_scatter_lane_ops_per_s; /* ds_or_b32 at random words of 64 KiB */
    double lds_read_lane_ops_per_s;       /* ds_read_b32, conflict-free */
    double lds_write_b64_bytes_per_s;     /* ds_write_b64, conflict-free, in bytes */
    double lds_or_wave_instr_per_s;       /* conflict-free ds_or_b32 wavefront instructions */
    double lds_or_half_lanes_wave_instr_per_s; /* the same with half the lanes masked off */
    double valu_wave_instr_per_s;         /* int32 add/xor wavefront instructions */
    double valu_wave_instr_per_clk_cu;    /* the same per CU per shader clock */
    double lds_or_clock_hz;               /* shader clock during the ds_or_b32 kernel */
    double valu_clock_hz;                 /* shader clock during the VALU kernel */
    uint32_t n_cu;
    uint32_t pad;
} sieve_peaks;

/* Run the microbenchmarks on the context's device (about 20 ms).  Errors:
 * SIEVE_EINVAL (NULL arguments), SIEVE_EDEVICE. */
SIEVE_API int sieve_measure_peaks(sieve_ctx *ctx, sieve_peaks *out);

/* ------------------------------------------------------------------------
 * Serving: a request loop with continuous batching.
 *
 * A server owns its own context on one device and a dispatcher thread.
 * Requests (ranges) are admitted in arrival order while their bitmaps get
 * room in two budgets that are real memory: a device pool of the HBM budget
 * (less the server's fixed device memory, allocated once at creation) and a
 * pinned host arena for the returned bitmaps.  Admitted requests are packed
 * into batches on up to `lanes` streams at once, so requests that arrive
 * while others run are batched and overlap on the device (the paper's
 * overlap of communication and computation, Section 2.2).  A batch of up to
 * 8 requests goes as plain range launches, one per request, on its lane's
 * stream; a larger one (or one with an empty or bucketed range) as one
 * launch of the sieve_batch work queue.  Results are identical to sieving
 * each range alone.
 * ---------------------------------------------------------------------- */
typedef struct sieve_server sieve_server;

#define SIEVE_SERVE_BATCHED 0u /* continuous batching over several lanes */
#define SIEVE_SERVE_PLAIN 1u   /* one request at a time, plain launches */

/* A zero field means the default in brackets. */
typedef struct sieve_server_config {
    uint32_t lanes;            /* batches in flight at once, one stream each [3] */
    uint32_t max_batch;        /* requests per batch [1024] */
    uint64_t max_batch_words;  /* bitmap words per batch, and the largest
                                  bitmap one request may ask for [2^26] */
    uint64_t hbm_budget_bytes; /* device bytes the server holds [32 GiB]: 64 MiB
                                  for its context (the full base-prime table),
                                  each lane's batch buffers (plain mode: the
                                  256 MiB hit-bucket pool), and the rest as the
                                  pool the admitted bitmaps live in */
    uint64_t host_arena_bytes; /* pinned host memory for returned bitmaps,
                                  held until released [2 GiB]; mapped into
                                  the device, where batched mode's copy
                                  kernels write them */
    uint32_t mode;             /* SIEVE_SERVE_BATCHED or SIEVE_SERVE_PLAIN */
    uint32_t pad;
} sieve_server_config;

/* A finished request.  words points into the server's pinned host arena
 * (flags & SIEVE_WANT_BITMAP) and stays valid until sieve_server_release.
 * Times are steady-clock nanoseconds. */
typedef struct sieve_result {
    uint64_t id;
    uint64_t lo;
    uint64_t hi;
    uint64_t pi;
    const uint32_t *words;
    uint64_t n_words;
    uint64_t t_submit_ns;
    uint64_t t_admit_ns;
    uint64_t t_launch_ns;
    uint64_t t_done_ns;
    int32_t status;
    uint32_t flags;
} sieve_result;

typedef struct sieve_server_stats {
    uint64_t submitted;
    uint64_t completed;
    uint64_t batches;           /* batches (or plain launches) issued */
    uint64_t single_launches;   /* batches of up to 8 requests served by plain
                                   range launches, one per request */
    uint64_t max_batch_seen;    /* most requests in one batch */
    uint64_t max_inflight;      /* most batches on the device at once */
    uint64_t deferred;          /* admissions that had to wait for budget */
    uint64_t peak_admitted_bytes; /* most device pool bytes held by admitted requests */
    uint64_t peak_host_bytes;   /* most pinned arena bytes held (until release) */
    uint64_t device_pool_bytes; /* size of the device bitmap pool */
    uint64_t graph_captures;    /* batch graphs captured after creation (0 unless a
                                   batch outgrew the buffers sized at creation) */
    uint64_t max_launch_call_ns; /* longest time the dispatcher spent queueing one
                                    batch or launch (host side) */
    uint64_t slow_launch_calls; /* such calls that took over 1 ms */
} sieve_server_stats;

/* Start a server on HIP device hip_device (cfg NULL = defaults).  Builds the
 * full base-prime table, allocates the device pool and the host arena and
 * captures each lane's batch graphs before returning.  Errors:
 * SIEVE_EINVAL, SIEVE_ENODEV, SIEVE_ENOMEM (also: the HBM budget does not
 * cover the fixed device memory), SIEVE_EDEVICE. */
SIEVE_API int sieve_server_create(int hip_device, const sieve_server_config *cfg, sieve_server **out);

/* Queue the range [lo, hi); flags: SIEVE_WANT_BITMAP to get its bitmap back.
 * Returns at once with the request id.  Errors: SIEVE_EINVAL (lo > hi, NULL
 * id_out), SIEVE_ERANGE (hi > SIEVE_MAX_HI), SIEVE_ENOMEM (its bitmap alone
 * exceeds max_batch_words or the largest block of the device pool or host
 * arena). */
SIEVE_API int sieve_server_submit(sieve_server *s, uint64_t lo, uint64_t hi, uint32_t flags,
                                  uint64_t *id_out);

/* Move up to max finished results into out[0 .. *n_out), waiting up to
 * wait_us microseconds for the first one. */
SIEVE_API int sieve_server_poll(sieve_server *s, sieve_result *out, uint32_t max, uint32_t *n_out,
                                uint32_t wait_us);

/* Return a finished bitmap request's host buffer to the arena.  Results
 * without a bitmap need no release.  SIEVE_EINVAL for an unknown id. */
SIEVE_API int sieve_server_release(sieve_server *s, uint64_t id);

SIEVE_API int sieve_server_get_stats(sieve_server *s, sieve_server_stats *out);

/* Finish every submitted request, stop the dispatcher and free everything
 * (unreleased result buffers included).  NULL is ignored. */
SIEVE_API int sieve_server_destroy(sieve_server *s);

/* Replay a timed trace through a server: request i (lo[i], hi[i],
 * flags[i]) is submitted at t_arrival_s[i] seconds after the start by a
 * native submitter thread; results are released as they arrive.  Fills
 * pi_out[i] and latency_ms_out[i] (from the scheduled arrival, start +
 * t_arrival_s[i], to the result on the host, so a submitter running late
 * counts as queueing), and stats_out if not NULL. */
SIEVE_API int sieve_serve_trace(int hip_device, const sieve_server_config *cfg, const uint64_t *lo,
                                const uint64_t *hi, const uint32_t *flags, const double *t_arrival_s,
                                uint64_t n, uint64_t *pi_out, double *latency_ms_out,
                                sieve_server_stats *stats_out);

#ifdef __cplusplus
}
#endif

#endif /* SIEVE_H */
