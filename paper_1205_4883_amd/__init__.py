"""Exact range sieve of Eratosthenes on AMD MI355X (gfx950).

The compute path is libsieve.so (hand-written HIP kernels behind the C ABI of
include/sieve.h); this package is its thin Python binding.
"""
from .sieve import (  # noqa: F401
    EXPORTED,
    INTERVAL_DTYPE,
    LIB_PATH,
    SIEVE_MAX_HI,
    Server,
    Sieve,
    SieveError,
    result_words,
    sieve_serve_trace,
    sieve_server_create,
    sieve_server_destroy,
    sieve_server_get_stats,
    sieve_server_poll,
    sieve_server_release,
    sieve_server_submit,
    sieve_autotune,
    sieve_base_primes,
    sieve_batch,
    sieve_bitmap_words,
    sieve_fermat_batch,
    sieve_is_prime_batch,
    sieve_create,
    sieve_destroy,
    sieve_get_tuning,
    sieve_last_hip_error,
    sieve_last_kernel_ms,
    sieve_plan,
    sieve_range_bitmap,
    sieve_range_count,
    sieve_set_timing,
    sieve_set_tuning,
    sieve_strerror,
)
