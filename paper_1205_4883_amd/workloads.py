"""Seeded synthetic inputs for the batched and served workloads.

Only random draws live here (no sieve arithmetic), so that the tests and the
bench see the same intervals.

batch_intervals(seed=0, n=4096)
    4096 intervals [a_i, a_i + L_i): a_i = floor(exp(U(ln 1e6, ln 1e12))),
    drawn as one vector, then L_i = floor(exp(U(ln 1e4, ln 1e8))).
serve_trace(seed=1, seconds=60.0, rate=2000.0)
    Poisson arrivals (exponential gaps, mean 1/rate s) until t >= seconds;
    then per request lo = floor(exp(U(ln 1e3, ln 1e12))),
    length = floor(exp(U(ln 1e3, ln 1e9))) and a bitmap flag ~ Bernoulli(0.5),
    each drawn as one vector in that order.
"""
import hashlib

import numpy as np


def _log_uniform_int(rng, lo, hi, n):
    return np.floor(np.exp(rng.uniform(np.log(lo), np.log(hi), n))).astype(np.uint64)


def batch_intervals(seed=0, n=4096):
    """(lo, hi) uint64 arrays of the batched workload."""
    rng = np.random.default_rng(seed)
    a = _log_uniform_int(rng, 1e6, 1e12, n)
    length = _log_uniform_int(rng, 1e4, 1e8, n)
    return a, a + length


def serve_trace(seed=1, seconds=60.0, rate=2000.0):
    """dict of arrays: t (s, float64), lo, hi (uint64), bitmap (bool)."""
    rng = np.random.default_rng(seed)
    gaps = []
    total = 0.0
    while total < seconds:
        g = rng.exponential(1.0 / rate, 65536)
        gaps.append(g)
        total += float(g.sum())
    t = np.cumsum(np.concatenate(gaps))
    t = t[t < seconds]
    n = t.size
    lo = _log_uniform_int(rng, 1e3, 1e12, n)
    length = _log_uniform_int(rng, 1e3, 1e9, n)
    bitmap = rng.random(n) < 0.5
    return {"t": t, "lo": lo, "hi": lo + length, "bitmap": bitmap}


def fingerprint(*arrays):
    """sha256 of the arrays' bytes, in order (little-endian as stored)."""
    h = hashlib.sha256()
    for a in arrays:
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()
