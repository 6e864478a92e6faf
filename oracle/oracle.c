/*
 * Oracle for the exact range sieve of Eratosthenes.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may load, call or
 * link this file: only the tests, the smoke check and the CPU-baseline leg of
 * the bench use it.  It shares no code, header or table with the HIP library.
 *
 * What it computes is the plain definition of the method's result (paper,
 * Section 1 and Section 3.1): the set of primes in a half-open integer range
 * [lo, hi), obtained by crossing off the multiples of every prime p with
 * p*p <= hi-1, and the size of that set, pi(hi-1) - pi(lo-1).  The paper's
 * own scheme (blocks spread over nodes, each block sifted from head and tail
 * by two cores, Eq. 3, Eq. 4, Alg. 1) only reorders the crossing-off, which
 * is an idempotent set operation, so every variant reaches this same set.
 *
 * Deliberately naive: one byte per odd integer, no wheel, no bit tricks, no
 * floating point.  Blocks of odd integers are handed to threads in contiguous
 * runs, ceil(nblocks / threads) each: the paper's block partition of Eq. 3
 * read as a ceiling (its printed form is garbled).
 *
 * Also here, for pinning and spot checks:
 *   - trial division (paper, Section 1: n is prime iff no prime <= sqrt(n)
 *     divides it);
 *   - modular exponentiation by repeated squaring (paper, Section 3.2,
 *     Alg. 2), with 128-bit products so that moduli up to 2^64 are exact;
 *   - the Fermat test (paper, Section 3.2, Alg. 3), with the random draws
 *     passed in by the caller;
 *   - deterministic Miller-Rabin, the stronger test the paper points to at the
 *     end of Section 3.2, with the first twelve primes as bases (exact for
 *     every 64-bit n).
 *
 * Output encoding of a range (the paper leaves it open): bit i of the bitmap
 * stands for the odd integer (lo with its low bit cleared) + 2*i + 1, for
 * i < floor(hi/2) - floor(lo/2); 32-bit little-endian words, least
 * significant bit first; 1 means prime; bits past the end are 0.  The even
 * prime 2 has no bit but is counted in pi when lo <= 2 < hi.
 */
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORACLE_OK 0
#define ORACLE_EINVAL (-1)
#define ORACLE_ERANGE (-2)
#define ORACLE_ENOMEM (-3)
#define ORACLE_EBUFSZ (-4)

/* Largest hi accepted: 10^15.  sqrt(10^15) < 2^25, so every base prime and
 * every intermediate product below stays far inside 64 bits. */
#define ORACLE_MAX_HI 1000000000000000ULL

/* Odd integers per block (one byte each). */
#define ORACLE_BLOCK_BITS (1u << 20)

/* floor(sqrt(n)) by bisection on r*r <= n; exact, no floating point. */
uint64_t oracle_isqrt(uint64_t n)
{
    uint64_t lo = 0, hi = 4294967296ULL; /* answer is in [lo, hi) */
    while (hi - lo > 1) {
        uint64_t mid = lo + (hi - lo) / 2;
        if (mid * mid <= n) /* mid < 2^32, so mid*mid cannot wrap */
            lo = mid;
        else
            hi = mid;
    }
    return lo;
}

/* Trial division (Section 1): n is prime iff n >= 2 and no d with
 * 2 <= d <= sqrt(n) divides it.  Dividing by every d rather than only the
 * primes gives the same answer and needs no prime table. */
int oracle_trial_division_is_prime(uint64_t n)
{
    if (n < 2)
        return 0;
    uint64_t r = oracle_isqrt(n);
    for (uint64_t d = 2; d <= r; d++)
        if (n % d == 0)
            return 0;
    return 1;
}

static uint64_t mulmod(uint64_t x, uint64_t y, uint64_t c)
{
    return (uint64_t)(((unsigned __int128)x * y) % c);
}

/* (a^b) mod c by repeated squaring (Section 3.2, Alg. 2): x accumulates the
 * product of the squares y = a^(2^k) for the set bits k of b.  The final
 * reduction makes c = 1 return 0.  c = 0 is undefined and returns 0. */
uint64_t oracle_modpow(uint64_t a, uint64_t b, uint64_t c)
{
    if (c == 0)
        return 0;
    uint64_t x = 1, y = a % c;
    while (b > 0) {
        if (b & 1)
            x = mulmod(x, y, c);
        y = mulmod(y, y, c);
        b >>= 1;
    }
    return x % c;
}

/* Fermat test (Section 3.2, Alg. 3).  The algorithm draws its bases at
 * random; here the caller passes the raw draws, and base i is
 * draws[i] mod (p-1) + 1 as in the paper.  Returns 1 for "probably prime". */
int oracle_fermat(uint64_t p, const uint64_t *draws, int iterations)
{
    if (p <= 1) /* the paper rejects p = 1; 0 is rejected the same way */
        return 0;
    if (p == 2) /* p-1 = 1: every base is 1, which passes */
        return 1;
    for (int i = 0; i < iterations; i++) {
        uint64_t a = draws[i] % (p - 1) + 1;
        if (oracle_modpow(a, p - 1, p) != 1)
            return 0;
    }
    return 1;
}

/* Deterministic Miller-Rabin for 64-bit n (the test the paper names as the
 * remedy for Carmichael numbers, end of Section 3.2).  Write n-1 = d*2^s with
 * d odd; a base a proves n composite unless a^d = 1 or a^(d*2^j) = n-1 for
 * some 0 <= j < s.  The first twelve primes as bases decide every n < 2^64
 * exactly (Sorenson and Webster, 2015). */
int oracle_mr_is_prime(uint64_t n)
{
    static const uint64_t bases[12] = {2, 3, 5, 7, 11, 13, 17, 19, 23, 29, 31, 37};
    if (n < 2)
        return 0;
    for (int i = 0; i < 12; i++) {
        if (n == bases[i])
            return 1;
        if (n % bases[i] == 0)
            return 0;
    }
    uint64_t d = n - 1;
    int s = 0;
    while ((d & 1) == 0) {
        d >>= 1;
        s++;
    }
    for (int i = 0; i < 12; i++) {
        uint64_t x = oracle_modpow(bases[i], d, n);
        if (x == 1 || x == n - 1)
            continue;
        int witness = 1;
        for (int j = 1; j < s; j++) {
            x = mulmod(x, x, n);
            if (x == n - 1) {
                witness = 0;
                break;
            }
        }
        if (witness)
            return 0;
    }
    return 1;
}

/* Plain sieve of Eratosthenes on [0, limit]: one byte per integer, crossing
 * off p*p, p*p + p, ... for each p still standing (Section 3.1).  Returns a
 * malloc'd array with is_prime[n] for 0 <= n <= limit, or NULL. */
static unsigned char *small_sieve(uint64_t limit)
{
    unsigned char *is_prime = (unsigned char *)malloc(limit + 1);
    if (!is_prime)
        return NULL;
    memset(is_prime, 1, limit + 1);
    is_prime[0] = 0;
    if (limit >= 1)
        is_prime[1] = 0;
    for (uint64_t p = 2; p * p <= limit; p++)
        if (is_prime[p])
            for (uint64_t m = p * p; m <= limit; m += p)
                is_prime[m] = 0;
    return is_prime;
}

/* Primes p <= limit, ascending.  With out == NULL or cap == 0 only *n_out is
 * set (size query).  limit must be <= sqrt(ORACLE_MAX_HI) rounded up. */
int oracle_base_primes(uint64_t limit, uint32_t *out, uint64_t cap, uint64_t *n_out)
{
    if (!n_out)
        return ORACLE_EINVAL;
    if (limit > 31622777ULL)
        return ORACLE_ERANGE;
    unsigned char *is_prime = small_sieve(limit);
    if (!is_prime)
        return ORACLE_ENOMEM;
    uint64_t n = 0;
    for (uint64_t k = 0; k <= limit; k++)
        n += is_prime[k];
    *n_out = n;
    if (out && cap) {
        if (cap < n) {
            free(is_prime);
            return ORACLE_EBUFSZ;
        }
        uint64_t j = 0;
        for (uint64_t k = 0; k <= limit; k++)
            if (is_prime[k])
                out[j++] = (uint32_t)k;
    }
    free(is_prime);
    return ORACLE_OK;
}

/* Number of odd integers (bitmap bits) in [lo, hi). */
uint64_t oracle_bitmap_bits(uint64_t lo, uint64_t hi)
{
    return hi / 2 - lo / 2;
}

uint64_t oracle_bitmap_words(uint64_t lo, uint64_t hi)
{
    return (oracle_bitmap_bits(lo, hi) + 31) / 32;
}

struct job {
    uint64_t first_odd;   /* the odd integer that bit 0 stands for */
    uint64_t nbits;       /* odd integers in the range */
    uint64_t blk_begin;   /* first block of this thread */
    uint64_t blk_end;     /* one past its last block */
    const uint32_t *primes; /* odd base primes, ascending */
    uint64_t n_primes;
    uint32_t *words;      /* output bitmap, or NULL for count only */
    uint64_t count;       /* primes found among the odd integers */
    int status;
};

static void *sieve_blocks(void *arg)
{
    struct job *jb = (struct job *)arg;
    unsigned char *a = (unsigned char *)malloc(ORACLE_BLOCK_BITS);
    if (!a) {
        jb->status = ORACLE_ENOMEM;
        return NULL;
    }
    uint64_t count = 0;
    for (uint64_t b = jb->blk_begin; b < jb->blk_end; b++) {
        uint64_t bit0 = b * ORACLE_BLOCK_BITS;
        uint64_t len = jb->nbits - bit0;
        if (len > ORACLE_BLOCK_BITS)
            len = ORACLE_BLOCK_BITS;
        /* a[j] stands for the odd integer f + 2j */
        uint64_t f = jb->first_odd + 2 * bit0;
        uint64_t end = f + 2 * len; /* first odd integer after the block */
        memset(a, 1, len);
        for (uint64_t i = 0; i < jb->n_primes; i++) {
            uint64_t p = jb->primes[i];
            /* first multiple of p that is >= f, and never below p*p */
            uint64_t m = (f + p - 1) / p * p;
            if (m < p * p)
                m = p * p;
            if (m % 2 == 0) /* even multiples are not in the bitmap */
                m += p;
            for (; m < end; m += 2 * p)
                a[(m - f) / 2] = 0;
        }
        if (f == 1) /* 1 is not prime */
            a[0] = 0;
        for (uint64_t j = 0; j < len; j++) {
            count += a[j];
            if (jb->words && a[j])
                jb->words[(bit0 + j) / 32] |= (uint32_t)1 << ((bit0 + j) % 32);
        }
    }
    free(a);
    jb->count = count;
    jb->status = ORACLE_OK;
    return NULL;
}

/*
 * The primes in [lo, hi): their count in *pi_out and, when words != NULL, the
 * odd-only bitmap in words[0 .. n_words).  threads >= 1 workers take
 * contiguous runs of blocks.
 * Errors: ORACLE_EINVAL (lo > hi, pi_out NULL, threads < 1),
 * ORACLE_ERANGE (hi > 10^15), ORACLE_EBUFSZ (n_words too small),
 * ORACLE_ENOMEM.
 */
int oracle_sieve_range(uint64_t lo, uint64_t hi, uint32_t *words, uint64_t n_words,
                       int threads, uint64_t *pi_out)
{
    if (!pi_out || lo > hi || threads < 1)
        return ORACLE_EINVAL;
    if (hi > ORACLE_MAX_HI)
        return ORACLE_ERANGE;
    uint64_t nbits = oracle_bitmap_bits(lo, hi);
    uint64_t nw = (nbits + 31) / 32;
    if (words) {
        if (n_words < nw)
            return ORACLE_EBUFSZ;
        memset(words, 0, n_words * sizeof(uint32_t));
    }
    uint64_t pi = (lo <= 2 && 2 < hi) ? 1 : 0;
    if (nbits == 0) {
        *pi_out = pi;
        return ORACLE_OK;
    }

    /* base primes: odd p with p*p <= hi - 1 */
    uint64_t r = oracle_isqrt(hi - 1);
    unsigned char *is_prime = small_sieve(r);
    if (!is_prime)
        return ORACLE_ENOMEM;
    uint64_t n_primes = 0;
    for (uint64_t k = 3; k <= r; k++)
        n_primes += is_prime[k];
    uint32_t *primes = (uint32_t *)malloc((n_primes + 1) * sizeof(uint32_t));
    if (!primes) {
        free(is_prime);
        return ORACLE_ENOMEM;
    }
    uint64_t j = 0;
    for (uint64_t k = 3; k <= r; k++)
        if (is_prime[k])
            primes[j++] = (uint32_t)k;
    free(is_prime);

    uint64_t nblocks = (nbits + ORACLE_BLOCK_BITS - 1) / ORACLE_BLOCK_BITS;
    if ((uint64_t)threads > nblocks)
        threads = (int)nblocks;
    uint64_t per = (nblocks + threads - 1) / threads; /* ceil, Eq. 3 */
    struct job *jobs = (struct job *)calloc(threads, sizeof(struct job));
    pthread_t *tid = (pthread_t *)calloc(threads, sizeof(pthread_t));
    if (!jobs || !tid) {
        free(jobs);
        free(tid);
        free(primes);
        return ORACLE_ENOMEM;
    }
    for (int t = 0; t < threads; t++) {
        jobs[t].first_odd = (lo & ~(uint64_t)1) + 1;
        jobs[t].nbits = nbits;
        jobs[t].blk_begin = (uint64_t)t * per;
        jobs[t].blk_end = jobs[t].blk_begin + per;
        if (jobs[t].blk_begin > nblocks)
            jobs[t].blk_begin = nblocks;
        if (jobs[t].blk_end > nblocks)
            jobs[t].blk_end = nblocks;
        jobs[t].primes = primes;
        jobs[t].n_primes = n_primes;
        jobs[t].words = words;
        jobs[t].status = ORACLE_EINVAL;
    }
    /* Blocks are a multiple of 32 bits, so threads never share a word. */
    int started = 0;
    for (int t = 1; t < threads; t++) {
        if (pthread_create(&tid[t], NULL, sieve_blocks, &jobs[t]) != 0)
            break;
        started = t;
    }
    sieve_blocks(&jobs[0]);
    for (int t = 1; t <= started; t++)
        pthread_join(tid[t], NULL);
    for (int t = started + 1; t < threads; t++) /* could not start: run here */
        sieve_blocks(&jobs[t]);
    int status = ORACLE_OK;
    for (int t = 0; t < threads; t++) {
        pi += jobs[t].count;
        if (jobs[t].status != ORACLE_OK)
            status = jobs[t].status;
    }
    free(jobs);
    free(tid);
    free(primes);
    if (status != ORACLE_OK)
        return status;
    *pi_out = pi;
    return ORACLE_OK;
}
