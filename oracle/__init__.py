"""CPU oracle for the exact range sieve: TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never loads it and
shares no code with it.

It wraps ``oracle.c`` (plain C, built into ``liboracle.so`` beside this file)
through ctypes.  Every function follows the plain definition of the method's
result (paper, Sections 1 and 3.1) or one of the paper's auxiliary
algorithms (Section 3.2, Algs. 2 and 3); the C file says which.
"""
import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")

OK, EINVAL, ERANGE, ENOMEM, EBUFSZ = 0, -1, -2, -3, -4
MAX_HI = 10**15

_lib = None


def build(force=True):
    """Compile oracle.c into liboracle.so with gcc (plain -O2, pthreads)."""
    if not force and os.path.exists(_LIB):
        return _LIB
    tmp = _LIB + ".tmp"
    subprocess.run(
        ["gcc", "-O2", "-std=c11", "-Wall", "-Wextra", "-shared", "-fPIC",
         "-pthread", _SRC, "-o", tmp],
        check=True,
    )
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    u64, u32p, u64p = ctypes.c_uint64, ctypes.POINTER(ctypes.c_uint32), ctypes.POINTER(ctypes.c_uint64)
    lib.oracle_isqrt.argtypes = [u64]
    lib.oracle_isqrt.restype = u64
    lib.oracle_trial_division_is_prime.argtypes = [u64]
    lib.oracle_trial_division_is_prime.restype = ctypes.c_int
    lib.oracle_modpow.argtypes = [u64, u64, u64]
    lib.oracle_modpow.restype = u64
    lib.oracle_fermat.argtypes = [u64, u64p, ctypes.c_int]
    lib.oracle_fermat.restype = ctypes.c_int
    lib.oracle_mr_is_prime.argtypes = [u64]
    lib.oracle_mr_is_prime.restype = ctypes.c_int
    lib.oracle_base_primes.argtypes = [u64, u32p, u64, u64p]
    lib.oracle_base_primes.restype = ctypes.c_int
    lib.oracle_bitmap_bits.argtypes = [u64, u64]
    lib.oracle_bitmap_bits.restype = u64
    lib.oracle_bitmap_words.argtypes = [u64, u64]
    lib.oracle_bitmap_words.restype = u64
    lib.oracle_sieve_range.argtypes = [u64, u64, u32p, u64, ctypes.c_int, u64p]
    lib.oracle_sieve_range.restype = ctypes.c_int
    _lib = lib
    return lib


class OracleError(RuntimeError):
    def __init__(self, status):
        super().__init__(f"oracle status {status}")
        self.status = status


def default_threads():
    return max(1, min(16, os.cpu_count() or 1))


def isqrt(n):
    return int(_load().oracle_isqrt(n))


def trial_division_is_prime(n):
    return bool(_load().oracle_trial_division_is_prime(n))


def modpow(a, b, c):
    return int(_load().oracle_modpow(a, b, c))


def fermat(p, draws):
    arr = (ctypes.c_uint64 * max(1, len(draws)))(*draws)
    return bool(_load().oracle_fermat(p, arr, len(draws)))


def mr_is_prime(n):
    return bool(_load().oracle_mr_is_prime(n))


def base_primes(limit):
    """Primes p <= limit ascending, as a numpy uint32 array."""
    lib = _load()
    n = ctypes.c_uint64(0)
    st = lib.oracle_base_primes(limit, None, 0, ctypes.byref(n))
    if st != OK:
        raise OracleError(st)
    out = np.zeros(max(1, n.value), dtype=np.uint32)
    st = lib.oracle_base_primes(
        limit, out.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), out.size, ctypes.byref(n))
    if st != OK:
        raise OracleError(st)
    return out[: n.value]


def bitmap_words(lo, hi):
    return int(_load().oracle_bitmap_words(lo, hi))


def count(lo, hi, threads=None):
    """pi over [lo, hi)."""
    pi = ctypes.c_uint64(0)
    st = _load().oracle_sieve_range(lo, hi, None, 0, threads or default_threads(), ctypes.byref(pi))
    if st != OK:
        raise OracleError(st)
    return pi.value


def bitmap(lo, hi, threads=None):
    """(words, pi): the odd-only prime bitmap of [lo, hi) as uint32 words."""
    lib = _load()
    nw = int(lib.oracle_bitmap_words(lo, hi))
    words = np.zeros(max(1, nw), dtype=np.uint32)
    pi = ctypes.c_uint64(0)
    st = lib.oracle_sieve_range(
        lo, hi, words.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)), words.size,
        threads or default_threads(), ctypes.byref(pi))
    if st != OK:
        raise OracleError(st)
    return words[:nw], pi.value


def status_of(lo, hi, n_words=None, words=True):
    """Status code the oracle returns for (lo, hi[, n_words]) without raising."""
    lib = _load()
    pi = ctypes.c_uint64(0)
    if words:
        buf = np.zeros(max(1, n_words or 1), dtype=np.uint32)
        return lib.oracle_sieve_range(
            lo, hi, buf.ctypes.data_as(ctypes.POINTER(ctypes.c_uint32)),
            n_words if n_words is not None else buf.size, 1, ctypes.byref(pi))
    return lib.oracle_sieve_range(lo, hi, None, 0, 1, ctypes.byref(pi))
