"""Thin ctypes binding of libsieve.so (include/sieve.h).

The functions carry the C names and only marshal arguments: every step of
the sieve runs in the library's HIP kernels.  PyTorch is used for device
memory (output tensors) and streams.  There is no fallback: if the library
is missing or no gfx950 device is present, the calls fail loudly.
"""
import ctypes
import os

import numpy as np

_PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_PKG, "libsieve.so")

SIEVE_OK = 0
SIEVE_EINVAL = -1
SIEVE_ERANGE = -2
SIEVE_ENOMEM = -3
SIEVE_EBUFSZ = -4
SIEVE_EDEVICE = -5
SIEVE_ENODEV = -6
SIEVE_EOVERFLOW = -7
SIEVE_MAX_HI = 10**15
SIEVE_WANT_BITMAP = 1

EXPORTED = [
    "sieve_create", "sieve_destroy", "sieve_strerror", "sieve_last_hip_error",
    "sieve_set_timing", "sieve_last_kernel_ms",
    "sieve_get_tuning", "sieve_set_tuning", "sieve_plan", "sieve_bitmap_words",
    "sieve_base_primes", "sieve_range_count", "sieve_range_bitmap", "sieve_batch",
    "sieve_range_bitmap_noalloc",
    "sieve_autotune", "sieve_is_prime_batch", "sieve_fermat_batch", "sieve_measure_peaks",
    "sieve_server_create", "sieve_server_submit", "sieve_server_poll", "sieve_server_release",
    "sieve_server_get_stats", "sieve_server_destroy", "sieve_serve_trace",
]

SIEVE_SERVE_BATCHED = 0
SIEVE_SERVE_PLAIN = 1


class sieve_tuning(ctypes.Structure):
    _fields_ = [("seg_bits", ctypes.c_uint32), ("dense_limit", ctypes.c_uint32),
                ("bucket_limit", ctypes.c_uint32), ("bucket_depth", ctypes.c_uint32),
                ("block_threads", ctypes.c_uint32), ("wg_per_cu", ctypes.c_uint32)]


class sieve_plan_info(ctypes.Structure):
    _fields_ = [("nbits", ctypes.c_uint64), ("n_words", ctypes.c_uint64),
                ("sqrt_bound", ctypes.c_uint64), ("n_segments", ctypes.c_uint64),
                ("seg_bits", ctypes.c_uint32), ("dense_limit", ctypes.c_uint32),
                ("block_threads", ctypes.c_uint32), ("bucket_limit", ctypes.c_uint32)]


class sieve_interval(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64),
                ("word_offset", ctypes.c_uint64), ("flags", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class sieve_peaks(ctypes.Structure):
    _fields_ = [("lds_or_lane_ops_per_s", ctypes.c_double), ("lds_or_lanes_per_clk_cu", ctypes.c_double),
                ("lds_write_lane_ops_per_s", ctypes.c_double),
                ("lds_or_scatter_lane_ops_per_s", ctypes.c_double),
                ("lds_read_lane_ops_per_s", ctypes.c_double), ("lds_write_b64_bytes_per_s", ctypes.c_double),
                ("lds_or_wave_instr_per_s", ctypes.c_double),
                ("lds_or_half_lanes_wave_instr_per_s", ctypes.c_double),
                ("valu_wave_instr_per_s", ctypes.c_double), ("valu_wave_instr_per_clk_cu", ctypes.c_double),
                ("lds_or_clock_hz", ctypes.c_double), ("valu_clock_hz", ctypes.c_double),
                ("n_cu", ctypes.c_uint32), ("pad", ctypes.c_uint32)]


class sieve_server_config(ctypes.Structure):
    _fields_ = [("lanes", ctypes.c_uint32), ("max_batch", ctypes.c_uint32),
                ("max_batch_words", ctypes.c_uint64), ("hbm_budget_bytes", ctypes.c_uint64),
                ("host_arena_bytes", ctypes.c_uint64), ("mode", ctypes.c_uint32),
                ("pad", ctypes.c_uint32)]


class sieve_result(ctypes.Structure):
    _fields_ = [("id", ctypes.c_uint64), ("lo", ctypes.c_uint64), ("hi", ctypes.c_uint64),
                ("pi", ctypes.c_uint64), ("words", ctypes.c_void_p), ("n_words", ctypes.c_uint64),
                ("t_submit_ns", ctypes.c_uint64), ("t_admit_ns", ctypes.c_uint64),
                ("t_launch_ns", ctypes.c_uint64), ("t_done_ns", ctypes.c_uint64),
                ("status", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class sieve_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_uint64), ("completed", ctypes.c_uint64),
                ("batches", ctypes.c_uint64), ("single_launches", ctypes.c_uint64),
                ("max_batch_seen", ctypes.c_uint64),
                ("max_inflight", ctypes.c_uint64), ("deferred", ctypes.c_uint64),
                ("peak_admitted_bytes", ctypes.c_uint64), ("peak_host_bytes", ctypes.c_uint64),
                ("device_pool_bytes", ctypes.c_uint64), ("graph_captures", ctypes.c_uint64),
                ("max_launch_call_ns", ctypes.c_uint64), ("slow_launch_calls", ctypes.c_uint64)]


INTERVAL_DTYPE = np.dtype([("lo", "<u8"), ("hi", "<u8"), ("word_offset", "<u8"),
                           ("flags", "<u4"), ("pad", "<u4")])
assert INTERVAL_DTYPE.itemsize == ctypes.sizeof(sieve_interval)


class SieveError(RuntimeError):
    def __init__(self, status, what=""):
        msg = _lib().sieve_strerror(status).decode() if _LIB else str(status)
        super().__init__(f"{what}: {msg} (status {status})" if what else f"{msg} (status {status})")
        self.status = status


_LIB = None


def _lib():
    global _LIB
    if _LIB is not None:
        return _LIB
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is not built; run __graft_entry__.build()")
    lib = ctypes.CDLL(LIB_PATH)
    u32, u64, vp, i32 = ctypes.c_uint32, ctypes.c_uint64, ctypes.c_void_p, ctypes.c_int
    u64p = ctypes.POINTER(ctypes.c_uint64)
    lib.sieve_create.argtypes = [ctypes.POINTER(vp), i32, u64]
    lib.sieve_destroy.argtypes = [vp]
    lib.sieve_strerror.argtypes = [i32]
    lib.sieve_strerror.restype = ctypes.c_char_p
    lib.sieve_last_hip_error.argtypes = [vp]
    lib.sieve_set_timing.argtypes = [vp, i32]
    lib.sieve_last_kernel_ms.argtypes = [vp, ctypes.POINTER(ctypes.c_double)]
    lib.sieve_get_tuning.argtypes = [vp, ctypes.POINTER(sieve_tuning)]
    lib.sieve_set_tuning.argtypes = [vp, ctypes.POINTER(sieve_tuning)]
    lib.sieve_plan.argtypes = [u64, u64, ctypes.POINTER(sieve_tuning), u32, u32,
                               ctypes.POINTER(sieve_plan_info)]
    lib.sieve_bitmap_words.argtypes = [u64, u64]
    lib.sieve_bitmap_words.restype = u64
    lib.sieve_base_primes.argtypes = [vp, u64, vp, u64, u64p]
    lib.sieve_range_count.argtypes = [vp, u64, u64, u64p, vp]
    lib.sieve_range_bitmap.argtypes = [vp, u64, u64, vp, u64, u64p, vp]
    lib.sieve_batch.argtypes = [vp, vp, u32, vp, u64, vp, vp]
    lib.sieve_range_bitmap_noalloc.argtypes = [vp, u64, u64, vp, u64, vp, vp]
    lib.sieve_is_prime_batch.argtypes = [vp, vp, u64, vp, vp]
    lib.sieve_fermat_batch.argtypes = [vp, vp, u64, vp, u32, vp, vp]
    lib.sieve_measure_peaks.argtypes = [vp, ctypes.POINTER(sieve_peaks)]
    lib.sieve_autotune.argtypes = [vp, vp, u32, u32, ctypes.POINTER(sieve_tuning),
                                    ctypes.POINTER(ctypes.c_double)]
    lib.sieve_server_create.argtypes = [i32, ctypes.POINTER(sieve_server_config), ctypes.POINTER(vp)]
    lib.sieve_server_submit.argtypes = [vp, u64, u64, u32, u64p]
    lib.sieve_server_poll.argtypes = [vp, ctypes.POINTER(sieve_result), u32, ctypes.POINTER(u32), u32]
    lib.sieve_server_release.argtypes = [vp, u64]
    lib.sieve_server_get_stats.argtypes = [vp, ctypes.POINTER(sieve_server_stats)]
    lib.sieve_server_destroy.argtypes = [vp]
    lib.sieve_serve_trace.argtypes = [i32, ctypes.POINTER(sieve_server_config), vp, vp, vp, vp, u64,
                                      vp, vp, ctypes.POINTER(sieve_server_stats)]
    for name in EXPORTED:
        if name not in ("sieve_strerror", "sieve_bitmap_words"):
            getattr(lib, name).restype = i32
    _LIB = lib
    return lib


def _check(status, what):
    if status != SIEVE_OK:
        raise SieveError(status, what)


# -- the C functions, same names -------------------------------------------

def sieve_create(hip_device=0, hbm_budget_bytes=0):
    ctx = ctypes.c_void_p()
    _check(_lib().sieve_create(ctypes.byref(ctx), hip_device, hbm_budget_bytes), "sieve_create")
    return ctx


def sieve_destroy(ctx):
    _check(_lib().sieve_destroy(ctx), "sieve_destroy")


def sieve_strerror(status):
    return _lib().sieve_strerror(status).decode()


def sieve_last_hip_error(ctx):
    return _lib().sieve_last_hip_error(ctx)


def sieve_set_timing(ctx, on):
    _check(_lib().sieve_set_timing(ctx, 1 if on else 0), "sieve_set_timing")


def sieve_last_kernel_ms(ctx):
    ms = ctypes.c_double(0.0)
    _check(_lib().sieve_last_kernel_ms(ctx, ctypes.byref(ms)), "sieve_last_kernel_ms")
    return ms.value


def sieve_get_tuning(ctx):
    t = sieve_tuning()
    _check(_lib().sieve_get_tuning(ctx, ctypes.byref(t)), "sieve_get_tuning")
    return {k: getattr(t, k) for k, _ in sieve_tuning._fields_}


def sieve_set_tuning(ctx, **fields):
    t = sieve_tuning(**fields)
    _check(_lib().sieve_set_tuning(ctx, ctypes.byref(t)), "sieve_set_tuning")


def sieve_plan(lo, hi, tuning=None, n_cu=256, lds_bytes=163840):
    info = sieve_plan_info()
    t = ctypes.byref(sieve_tuning(**tuning)) if tuning else None
    _check(_lib().sieve_plan(lo, hi, t, n_cu, lds_bytes, ctypes.byref(info)), "sieve_plan")
    return {k: getattr(info, k) for k, _ in sieve_plan_info._fields_}


def sieve_bitmap_words(lo, hi):
    return int(_lib().sieve_bitmap_words(lo, hi))


def sieve_base_primes(ctx, limit):
    """All primes <= limit (computed on the device) as a numpy uint32 array."""
    n = ctypes.c_uint64(0)
    _check(_lib().sieve_base_primes(ctx, limit, None, 0, ctypes.byref(n)), "sieve_base_primes")
    out = np.zeros(max(1, n.value), dtype=np.uint32)
    _check(_lib().sieve_base_primes(ctx, limit, out.ctypes.data, out.size, ctypes.byref(n)),
           "sieve_base_primes")
    return out[: n.value]


def _stream_ptr(stream):
    if stream is None:
        return None
    return ctypes.c_void_p(stream if isinstance(stream, int) else stream.cuda_stream)


def sieve_range_count(ctx, lo, hi, stream=None):
    pi = ctypes.c_uint64(0)
    _check(_lib().sieve_range_count(ctx, lo, hi, ctypes.byref(pi), _stream_ptr(stream)),
           "sieve_range_count")
    return pi.value


def sieve_range_bitmap(ctx, lo, hi, d_words, n_words, want_pi=True, stream=None):
    """d_words: device address (int) or a CUDA tensor; returns pi or None."""
    ptr = d_words.data_ptr() if hasattr(d_words, "data_ptr") else d_words
    pi = ctypes.c_uint64(0)
    _check(_lib().sieve_range_bitmap(ctx, lo, hi, ctypes.c_void_p(ptr), n_words,
                                     ctypes.byref(pi) if want_pi else None, _stream_ptr(stream)),
           "sieve_range_bitmap")
    return pi.value if want_pi else None


def sieve_range_bitmap_noalloc(ctx, lo, hi, d_words, n_words, d_pi, stream=None):
    """The allocation-free call: d_words (bitmap, or None to count only) and
    d_pi (one int64 element receiving pi, or None) are device tensors or
    addresses, written in stream order; nothing is allocated or waited on."""
    _check(_lib().sieve_range_bitmap_noalloc(ctx, lo, hi, ctypes.c_void_p(_ptr(d_words)), n_words,
                                             ctypes.c_void_p(_ptr(d_pi)), _stream_ptr(stream)),
           "sieve_range_bitmap_noalloc")


def sieve_batch(ctx, intervals, d_words=None, total_words=0, stream=None):
    """intervals: numpy array of INTERVAL_DTYPE.  Returns numpy uint64 pi per interval."""
    iv = np.ascontiguousarray(intervals, dtype=INTERVAL_DTYPE)
    pi = np.zeros(max(1, len(iv)), dtype=np.uint64)
    ptr = d_words.data_ptr() if hasattr(d_words, "data_ptr") else (d_words or 0)
    _check(_lib().sieve_batch(ctx, iv.ctypes.data, len(iv), ctypes.c_void_p(ptr), total_words,
                              pi.ctypes.data, _stream_ptr(stream)), "sieve_batch")
    return pi[: len(iv)]


def _ptr(x):
    return x.data_ptr() if hasattr(x, "data_ptr") else (x or 0)


def sieve_is_prime_batch(ctx, d_n, count, d_out, stream=None):
    """Device arrays: d_n uint64[count] -> d_out uint8[count] (1 = prime)."""
    _check(_lib().sieve_is_prime_batch(ctx, ctypes.c_void_p(_ptr(d_n)), count,
                                       ctypes.c_void_p(_ptr(d_out)), _stream_ptr(stream)),
           "sieve_is_prime_batch")


def sieve_fermat_batch(ctx, d_n, count, d_draws, iterations, d_out, stream=None):
    """Alg. 3 on device arrays, with the caller's random draws."""
    _check(_lib().sieve_fermat_batch(ctx, ctypes.c_void_p(_ptr(d_n)), count,
                                     ctypes.c_void_p(_ptr(d_draws)), iterations,
                                     ctypes.c_void_p(_ptr(d_out)), _stream_ptr(stream)),
           "sieve_fermat_batch")


def sieve_measure_peaks(ctx):
    """Measured LDS and VALU peaks of the context's device (a dict)."""
    pk = sieve_peaks()
    _check(_lib().sieve_measure_peaks(ctx, ctypes.byref(pk)), "sieve_measure_peaks")
    return {k: getattr(pk, k) for k, _ in sieve_peaks._fields_ if k != "pad"}


SIEVE_TUNE_APPLY = 1
SIEVE_TUNE_FORCE = 2


def sieve_autotune(ctx, los, his=None, apply=True, force=False):
    """Time candidate tunings on the ranges [los[i], his[i]) (count only), or
    on `los` given as an INTERVAL_DTYPE array (his None), whose bitmap flags
    and word offsets are kept; returns (tuning dict, kernel ms of the winner)."""
    if his is None:
        iv = np.ascontiguousarray(los, dtype=INTERVAL_DTYPE)
    else:
        los = np.atleast_1d(np.asarray(los, dtype=np.uint64))
        his = np.atleast_1d(np.asarray(his, dtype=np.uint64))
        iv = np.zeros(len(los), dtype=INTERVAL_DTYPE)
        iv["lo"], iv["hi"] = los, his
    t = sieve_tuning()
    ms = ctypes.c_double(0)
    flags = (SIEVE_TUNE_APPLY if apply else 0) | (SIEVE_TUNE_FORCE if force else 0)
    _check(_lib().sieve_autotune(ctx, iv.ctypes.data, len(iv), flags, ctypes.byref(t),
                                 ctypes.byref(ms)), "sieve_autotune")
    return {k: getattr(t, k) for k, _ in sieve_tuning._fields_}, ms.value


def _server_config(cfg):
    c = sieve_server_config()
    for k, v in (cfg or {}).items():
        setattr(c, k, v)
    return c


def sieve_server_create(hip_device=0, **cfg):
    srv = ctypes.c_void_p()
    c = _server_config(cfg)
    _check(_lib().sieve_server_create(hip_device, ctypes.byref(c), ctypes.byref(srv)),
           "sieve_server_create")
    return srv


def sieve_server_submit(srv, lo, hi, flags=0):
    rid = ctypes.c_uint64(0)
    _check(_lib().sieve_server_submit(srv, lo, hi, flags, ctypes.byref(rid)), "sieve_server_submit")
    return rid.value


def sieve_server_poll(srv, max_results=256, wait_us=0):
    """Finished results as dicts; 'words' is the host address of a bitmap
    result (release it with sieve_server_release) or 0."""
    buf = (sieve_result * max(1, max_results))()
    n = ctypes.c_uint32(0)
    _check(_lib().sieve_server_poll(srv, buf, max_results, ctypes.byref(n), wait_us),
           "sieve_server_poll")
    return [{k: getattr(buf[i], k) or 0 for k, _ in sieve_result._fields_} for i in range(n.value)]


def result_words(result):
    """Copy of a bitmap result's words as a numpy uint32 array."""
    if not result["words"]:
        return np.zeros(0, dtype=np.uint32)
    arr = (ctypes.c_uint32 * result["n_words"]).from_address(result["words"])
    return np.frombuffer(arr, dtype=np.uint32).copy()


def sieve_server_release(srv, rid):
    _check(_lib().sieve_server_release(srv, rid), "sieve_server_release")


def sieve_server_get_stats(srv):
    st = sieve_server_stats()
    _check(_lib().sieve_server_get_stats(srv, ctypes.byref(st)), "sieve_server_get_stats")
    return {k: getattr(st, k) for k, _ in sieve_server_stats._fields_}


def sieve_server_destroy(srv):
    _check(_lib().sieve_server_destroy(srv), "sieve_server_destroy")


def sieve_serve_trace(hip_device, lo, hi, flags, t_arrival_s, **cfg):
    """Replay a timed trace natively; returns (pi, latency_ms, stats)."""
    lo = np.ascontiguousarray(lo, dtype=np.uint64)
    hi = np.ascontiguousarray(hi, dtype=np.uint64)
    flags = np.ascontiguousarray(flags, dtype=np.uint32)
    t = np.ascontiguousarray(t_arrival_s, dtype=np.float64)
    n = lo.size
    pi = np.zeros(max(1, n), dtype=np.uint64)
    lat = np.zeros(max(1, n), dtype=np.float64)
    st = sieve_server_stats()
    c = _server_config(cfg)
    _check(_lib().sieve_serve_trace(hip_device, ctypes.byref(c), lo.ctypes.data, hi.ctypes.data,
                                    flags.ctypes.data, t.ctypes.data, n, pi.ctypes.data,
                                    lat.ctypes.data, ctypes.byref(st)), "sieve_serve_trace")
    return pi[:n], lat[:n], {k: getattr(st, k) for k, _ in sieve_server_stats._fields_}


class Server:
    """A serving loop on one GPU; results come back as numpy arrays."""

    def __init__(self, device=0, **cfg):
        self.srv = sieve_server_create(device, **cfg)

    def submit(self, lo, hi, bitmap=False):
        return sieve_server_submit(self.srv, lo, hi, SIEVE_WANT_BITMAP if bitmap else 0)

    def results(self, wait_us=1000):
        """Finished results: dicts with 'id', 'pi', 'words' (numpy or None), timings."""
        out = []
        for r in sieve_server_poll(self.srv, 256, wait_us):
            words = None
            if r["words"]:
                words = result_words(r)
                sieve_server_release(self.srv, r["id"])
            r = dict(r, words=words)
            out.append(r)
        return out

    def stats(self):
        return sieve_server_get_stats(self.srv)

    def close(self):
        if self.srv is not None:
            sieve_server_destroy(self.srv)
            self.srv = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


# -- convenience wrapper over torch tensors -----------------------------------

class Sieve:
    """A context on one GPU; outputs are torch tensors on that device."""

    def __init__(self, device=0, hbm_budget_bytes=0):
        import torch

        self.torch = torch
        self.device = device
        self.ctx = sieve_create(device, hbm_budget_bytes)

    def close(self):
        if self.ctx is not None:
            sieve_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _stream(self):
        return self.torch.cuda.current_stream(self.device)

    def tuning(self, **fields):
        if fields:
            sieve_set_tuning(self.ctx, **fields)
        return sieve_get_tuning(self.ctx)

    def base_primes(self, limit):
        return sieve_base_primes(self.ctx, limit)

    def _u64_tensor(self, ns):
        arr = np.ascontiguousarray(np.asarray(ns, dtype=np.uint64))
        t = self.torch.from_numpy(arr.view(np.int64)).to(f"cuda:{self.device}")
        return arr, t

    def is_prime(self, ns):
        """numpy bool array: primality of each uint64 in ns (on the GPU)."""
        arr, d_n = self._u64_tensor(ns)
        out = self.torch.empty(max(1, arr.size), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        sieve_is_prime_batch(self.ctx, d_n, arr.size, out, stream=self._stream())
        return out[: arr.size].cpu().numpy().astype(bool)

    def fermat(self, ns, draws):
        """numpy bool array: the Fermat test (Alg. 3) of each n with the given draws."""
        arr, d_n = self._u64_tensor(ns)
        _, d_draws = self._u64_tensor(draws if len(draws) else [0])
        out = self.torch.empty(max(1, arr.size), dtype=self.torch.uint8, device=f"cuda:{self.device}")
        sieve_fermat_batch(self.ctx, d_n, arr.size, d_draws, len(draws), out, stream=self._stream())
        return out[: arr.size].cpu().numpy().astype(bool)

    def count(self, lo, hi):
        return sieve_range_count(self.ctx, lo, hi, stream=self._stream())

    def alloc_words(self, lo, hi):
        n = sieve_bitmap_words(lo, hi)
        return self.torch.empty(max(1, n), dtype=self.torch.int32, device=f"cuda:{self.device}")

    def bitmap(self, lo, hi, out=None, want_pi=True):
        """(words tensor, pi).  words is int32 with the layout of sieve.h."""
        n = sieve_bitmap_words(lo, hi)
        if out is None:
            out = self.alloc_words(lo, hi)
        pi = sieve_range_bitmap(self.ctx, lo, hi, out, out.numel(), want_pi, stream=self._stream())
        return out[:n], pi

    def batch(self, los, his, want_bitmap=False, out=None):
        """Per-interval pi (numpy uint64) and, with want_bitmap, (words, offsets)."""
        los = np.asarray(los, dtype=np.uint64)
        his = np.asarray(his, dtype=np.uint64)
        iv = np.zeros(len(los), dtype=INTERVAL_DTYPE)
        iv["lo"], iv["hi"] = los, his
        words = None
        total = 0
        if want_bitmap:
            nw = his // 2 - los // 2
            nw = (nw + 31) // 32
            offs = np.zeros(len(los), dtype=np.uint64)
            if len(los):
                offs[1:] = np.cumsum(nw)[:-1]
            total = int(nw.sum())
            iv["word_offset"] = offs
            iv["flags"] = SIEVE_WANT_BITMAP
            words = out if out is not None else self.torch.empty(
                max(1, total), dtype=self.torch.int32, device=f"cuda:{self.device}")
        pi = sieve_batch(self.ctx, iv, words, words.numel() if words is not None else 0,
                         stream=self._stream())
        if want_bitmap:
            return pi, words, iv["word_offset"].copy()
        return pi
