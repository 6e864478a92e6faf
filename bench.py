"""Benchmark: exact sieve of Eratosthenes on one MI355X.

Default workload: the count-only sieve of [2, 1e10) (pi = 455052511), one
step = one sieve_range_count call (base primes resident, pre-sieve, dense and
sparse marking, popcount reduction, count published to pinned memory).
Prints one JSON line.  Besides the headline it carries a block per other
workload: c1 and c2 (the bitmaps of [2, 1e7) and [2, 1e9)), batch (4096
intervals in one graph launch, autotuned, against 4096 plain calls), serve
(the 60 s Poisson trace through the serving loop, batched and plain) and mr
(batched Miller-Rabin).

  python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME]

Workloads: count-1e10 (default), bitmap-1e9, bitmap-1e7 (one range per
step), batch-4096 (4096 seeded intervals per sieve_batch call), serve-2000
(the 60 s trace), mr-2e24 (Miller-Rabin of 2^24 random odd 64-bit integers).

Throughput is sieved integers per second, (hi - lo) / step time.  The roofline
object prices the marking kernel's algorithmic LDS work against the LDS
atomic-OR rate measured on this device by sieve_measure_peaks (the planning
figure, 256 CUs x 32 banks x 2.4 GHz, beside it).  The work is one 32-bit LDS
atomic per crossed-off odd multiple m of every base prime 37 <= p <=
sqrt(hi-1), max(p^2, lo) <= m < hi (the kernels strike 3..31 with periodic
pre-sieve tables), plus one LDS write and one read per bitmap word;
issued_frac prices the atomics the kernels actually issue (multipliers prime
to 30) plus their per-word LDS accesses.  The wheel-30 work (marks from p = 7,
which a build pre-sieving only 3 and 5 would do) is in work_per_launch for
comparison; it is not priced, since this build strikes 7..31 with tables.  Its `units`
object gives each unit's use from the committed rocprofv3 counters of the
same kernel source (VALU issue against the measured VALU peak, LDS busy and
bank-conflict cycles), and `bound` names the busier one.  The cpu_baseline
object times the CPU oracle on the host over the same range.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "sieved ints/s on [2,1e10] (% roofline); batched vs plain speedup; p50/p99 ms"

WORKLOADS = {
    "bitmap-1e7": dict(lo=2, hi=10**7, bitmap=True, pi=664579,
               name="plain sieve of [2, 1e7): odd-only bitmap to HBM plus pi"),
    "bitmap-1e9": dict(lo=2, hi=10**9, bitmap=True, pi=50847534,
               name="plain sieve of [2, 1e9): odd-only bitmap (62.5 MB) to HBM plus pi"),
    "count-1e10": dict(lo=2, hi=10**10, bitmap=False, pi=455052511,
               name="count-only segmented sieve of [2, 1e10)"),
}

# MI355X: 256 CUs at 2.4 GHz; 32 LDS banks of 4 bytes per CU, one 32-bit
# lane access per bank per clock.
N_CU, CLOCK_HZ, LDS_LANES_PER_CLK = 256, 2.4e9, 32
LDS_PEAK_LANE_OPS = N_CU * CLOCK_HZ * LDS_LANES_PER_CLK
HBM_PEAK_BPS = 8.0e12


def device_info(torch):
    """Name, architecture and compute-unit count as the runtime reports them.
    The shader clock the kernels ran at is in `peaks` (measured by the
    microbenchmarks' own cycle and wall counters) and in the roofline's
    units (kernel cycles from the committed counters over the kernel time)."""
    props = torch.cuda.get_device_properties(0)
    return {"name": props.name, "gcn_arch": getattr(props, "gcnArchName", ""),
            "compute_units": props.multi_processor_count}


def host_info(threads):
    """Host CPU model, logical CPUs visible to this process, oracle threads."""
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mhz = []
    try:
        with open("/proc/cpuinfo") as f:
            mhz = [float(line.split(":", 1)[1]) for line in f if line.startswith("cpu MHz")]
    except (OSError, ValueError):
        pass
    return {"cpu_model": model, "nproc": len(os.sched_getaffinity(0)), "threads": threads,
            "cpu_mhz_mean": round(sum(mhz) / len(mhz), 1) if mhz else None}


# Odd primes the segment kernels strike with periodic pre-sieve tables instead
# of marking; crossing off starts at the next prime.
PRESIEVE_PRIMES = [3, 5, 7, 11, 13, 17, 19, 23, 29, 31]
FIRST_MARKED_PRIME = 37


def _odd_multiples(p, lo, hi):
    """Per prime p: the odd multiples m of p with max(p^2, lo) <= m < hi."""
    import numpy as np

    a = np.maximum(p * p, lo)
    jhi = (hi - 1) // p          # largest multiplier with m < hi
    jlo = -(-a // p)             # smallest multiplier with m >= a
    odd_upto = lambda x: (x + 1) // 2  # odd j in [1, x]
    return np.maximum(odd_upto(jhi) - odd_upto(jlo - 1), 0)


# Multipliers m prime to 30: the wheel the marking kernels walk (3 | m or
# 5 | m is struck by the pre-sieve).  _WHEEL_UPTO[r] = such m in [1, r].
_WHEEL = (1, 7, 11, 13, 17, 19, 23, 29)
_WHEEL_UPTO = [sum(1 for w in _WHEEL if w <= r) for r in range(30)]


def _wheel_multiples(p, lo, hi):
    """Per prime p: the multiples p*m, m prime to 30, with max(p^2, lo) <= p*m
    < hi -- the LDS atomics the marking kernels issue for p."""
    import numpy as np

    def upto(x):  # multipliers prime to 30 in [1, x]
        x = np.maximum(x, 0)
        return 8 * (x // 30) + np.asarray(_WHEEL_UPTO, dtype=np.int64)[x % 30]

    a = np.maximum(p * p, lo)
    mhi = (hi - 1) // p
    mlo = -(-a // p)
    return np.maximum(upto(mhi) - upto(mlo - 1), 0)


# LDS accesses per bitmap word besides the marks: the pre-sieve's three
# table reads and its store, and the count's read.
ISSUED_OPS_PER_WORD = 5


def algorithmic_lds_ops(primes, lo, hi, pmin=FIRST_MARKED_PRIME):
    """Marks (odd multiples m of each base prime pmin <= p <= isqrt(hi-1) with
    max(p^2, lo) <= m < hi) plus two LDS accesses per bitmap word (the
    pre-sieve write and the count read).  With pmin = 37 this is the work of
    this build, whose pre-sieve covers 3..31; pmin = 7 gives the wheel-30
    count (only 3 and 5 pre-sieved)."""
    import numpy as np

    p = np.asarray(primes).astype(np.int64)
    p = p[(p >= pmin) & (p * p <= hi - 1)]
    marks = int(_odd_multiples(p, lo, hi).sum())
    words = (hi // 2 - lo // 2 + 31) // 32
    return marks, marks + 2 * words, words


def lds_roofline(primes, ranges, seconds):
    """LDS roofline object for one launch that sieves `ranges` in `seconds`:
    frac prices this build's own work (marks of primes from 37 up), and
    issued_frac the atomics and per-word accesses the kernels issue; the
    wheel-30 work (marks from 7 up) is reported beside them, not priced."""
    import math

    import numpy as np

    p = np.asarray(primes).astype(np.int64)
    p = p[p >= 7]
    n_pre = int(np.searchsorted(p, FIRST_MARKED_PRIME))  # 7..31, struck by the pre-sieve
    marks = marks30 = words = 0
    ranges_list = [(int(a), int(b)) for a, b in ranges]
    for lo, hi in ranges_list:
        if hi <= lo:
            continue
        k = int(np.searchsorted(p, math.isqrt(hi - 1), side="right")) if hi > 1 else 0
        per = _odd_multiples(p[:k], lo, hi)
        m30 = int(per.sum())
        marks30 += m30
        marks += m30 - int(per[:n_pre].sum())
        words += (hi // 2 - lo // 2 + 31) // 32
    lane_ops, lane_ops30 = marks + 2 * words, marks30 + 2 * words
    issued = issued_marks(p[n_pre:], ranges_list)
    issued_ops = issued + ISSUED_OPS_PER_WORD * words
    achieved = lane_ops / seconds
    return {
        "bound": "lds", "achieved": achieved / 1e9, "peak": LDS_PEAK_LANE_OPS / 1e9,
        "unit": "Glane-op/s", "frac": achieved / LDS_PEAK_LANE_OPS,
        "issued_frac": issued_ops / seconds / LDS_PEAK_LANE_OPS,
        "work_per_launch": {"marks": marks, "lds_lane_ops": lane_ops, "words": words,
                            "first_marked_prime": FIRST_MARKED_PRIME,
                            "marks_wheel30": marks30, "lds_lane_ops_wheel30": lane_ops30,
                            "issued_marks": issued, "issued_lds_lane_ops": issued_ops}}


def issued_marks(p, ranges):
    """The LDS atomics the marking kernels issue: multiples p*m with m prime
    to 30, from max(p^2, lo), for the marking primes p (>= 37) of each range."""
    import math

    import numpy as np

    total = 0
    for lo, hi in ranges:
        if hi <= lo:
            continue
        k = int(np.searchsorted(p, math.isqrt(hi - 1), side="right")) if hi > 1 else 0
        total += int(_wheel_multiples(p[:k], lo, hi).sum())
    return total


def kernel_source_hash():
    """sha256/16 of the code of the kernel sources: line comments, trailing
    blanks and empty lines are dropped, so a comment edit does not make the
    committed counter runs stale."""
    h = hashlib.sha256()
    for f in ["sieve_kernels.hip", "sieve_internal.h"]:
        with open(os.path.join(ROOT, "paper_1205_4883_amd", "csrc", f), encoding="utf-8") as fh:
            for line in fh:
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()[:16]


def load_traffic(workload):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec.get("hbm_bytes_per_launch")


def load_counters(workload):
    """Per-dispatch rocprofv3 counters of the workload's dominant kernel from
    the committed profile, if taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", f"counters_{workload}.json")
    if not os.path.exists(path):
        return None
    with open(path) as f:
        rec = json.load(f)
    if rec.get("kernel_source_sha256_16") != kernel_source_hash():
        return None
    return rec


def unit_use(counters, peaks, n_cu, kernel_ms):
    """Each unit's use during the kernel from its counters: VALU issue
    (wave-instructions per clock per CU) against the measured VALU peak, and
    the fraction of cycles the LDS was busy (and how much of that was bank
    conflicts).  `bound` is the busier unit."""
    if not counters:
        return None, {"note": "no counters for the current kernel source"}
    c = counters["per_dispatch"]
    cycles = c["GRBM_GUI_ACTIVE"] / 8.0  # the counter sums the eight XCDs
    valu_clk = c["SQ_INSTS_VALU"] / n_cu / cycles
    valu_peak = peaks["valu_wave_instr_per_clk_cu"] if peaks else 1.0
    lds_busy = c["SQ_LDS_IDX_ACTIVE"] / n_cu / cycles
    units = {
        "valu": {"wave_instr_per_clk_cu": valu_clk, "peak_per_clk_cu": valu_peak,
                 "frac": valu_clk / valu_peak, "instr_per_dispatch": c["SQ_INSTS_VALU"]},
        "lds": {"busy_frac": lds_busy,
                "bank_conflict_share_of_busy": c["SQ_LDS_BANK_CONFLICT"] / c["SQ_LDS_IDX_ACTIVE"],
                "instr_per_dispatch": c["SQ_INSTS_LDS"]},
        "kernel_clock_hz_from_counters": cycles / (counters["kernel_ns_avg"] * 1e-9),
        "counters_kernel_ms": counters["kernel_ns_avg"] * 1e-6,
        "source": f"profiles/counters_{counters['workload']}.json",
    }
    bound = "valu" if units["valu"]["frac"] > lds_busy else "lds"
    return bound, units


def measured_roofline(primes, ranges, seconds, peaks, counters, workload_key, kernel_name):
    """lds_roofline against the measured LDS atomic-OR peak (planning peak
    beside it), with the units' use from the counters and the binding unit."""
    roof = lds_roofline(primes, ranges, seconds)
    if peaks:
        measured = peaks["lds_or_lane_ops_per_s"]
        roof["frac_planning_peak"] = roof["frac"]
        roof["peak_planning"] = roof["peak"]
        roof["peak"] = measured / 1e9
        roof["frac"] = roof["achieved"] * 1e9 / measured
        roof["issued_frac"] = roof["issued_frac"] * LDS_PEAK_LANE_OPS / measured
        roof["peak_source"] = "measured: conflict-free ds_or_b32 on every CU (sieve_measure_peaks)"
    bound, units = unit_use(counters, peaks, N_CU, seconds * 1e3)
    roof["bound"] = bound or "lds"
    roof["units"] = units
    roof["traffic"] = load_traffic(workload_key)
    roof["kernel"] = kernel_name
    return roof


def run_single(sv, torch, s, wl, steps, warmup, peaks, workload_key, latency_calls=0):
    """One range per step: kernel time from HIP events (timing on), then the
    call time as production uses it (timing off).  Returns the record."""
    import numpy as np

    lo, hi = wl["lo"], wl["hi"]
    stream = torch.cuda.current_stream(0)
    out = s.alloc_words(lo, hi) if wl["bitmap"] else None

    def step():
        if out is None:
            return sv.sieve_range_count(s.ctx, lo, hi, stream=stream)
        return sv.sieve_range_bitmap(s.ctx, lo, hi, out, out.numel(), True, stream=stream)

    sv.sieve_set_timing(s.ctx, True)
    t_cold = time.perf_counter()
    assert step() == wl["pi"]  # cold: base primes beyond the context's table, plans
    torch.cuda.synchronize()
    cold_ms = 1e3 * (time.perf_counter() - t_cold)
    for _ in range(warmup):
        assert step() == wl["pi"]
    kernel_ms = []
    for _ in range(max(steps, 20)):
        assert step() == wl["pi"]
        kernel_ms.append(sv.sieve_last_kernel_ms(s.ctx))
    sv.sieve_set_timing(s.ctx, False)  # calls as in production, no events
    torch.cuda.synchronize()
    n_calls = max(steps, latency_calls)
    call_ms = []
    t0 = time.perf_counter()
    for _ in range(n_calls):
        tc = time.perf_counter()
        pi = step()
        call_ms.append(1e3 * (time.perf_counter() - tc))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / n_calls
    assert pi == wl["pi"], pi
    primes = sv.sieve_base_primes(s.ctx, int(np.sqrt(hi)) + 1)
    k_ms = float(np.mean(kernel_ms))
    plan = sv.sieve_plan(lo, hi, tuning=s.tuning())
    roof = measured_roofline(primes, [(lo, hi)], k_ms * 1e-3, peaks, load_counters(workload_key),
                             workload_key, "range_kernel<write=%s>" % ("true" if wl["bitmap"] else "false"))
    roof.update({"kernel_ms": k_ms, "kernel_ms_min": float(np.min(kernel_ms))})
    if wl["bitmap"]:
        words = roof["work_per_launch"]["words"]
        roof["hbm_write_GBps"] = 4 * words / (k_ms * 1e-3) / 1e9
        roof["hbm_write_frac"] = roof["hbm_write_GBps"] * 1e9 / HBM_PEAK_BPS
    return {
        "workload": wl["name"], "lo": lo, "hi": hi, "pi": pi, "calls": n_calls,
        "ms_per_call": 1e3 * dt, "ints_per_s": (hi - lo) / dt, "cold_ms": cold_ms,
        "call_ms": {"p50": float(np.percentile(call_ms, 50)), "min": float(np.min(call_ms)),
                    "p99": float(np.percentile(call_ms, 99)), "max": float(np.max(call_ms))},
        "plan": {k: plan[k] for k in ("seg_bits", "dense_limit", "block_threads", "n_segments")},
        "roofline": roof,
    }


def run_batch(sv, torch, s, steps, warmup, check_plain=True, tune=True, peaks=None):
    """The batched workload: 4096 seeded intervals, per-interval pi and packed
    bitmaps from one sieve_batch call (one graph launch), against the same
    intervals sieved one sieve_range_bitmap call at a time on one stream.
    With tune, sieve_autotune picks the segment size, dense bound and
    workgroups per CU on these intervals (bitmaps included) first and the
    context keeps its choice; the automatic plan is one of its candidates."""
    import numpy as np

    from paper_1205_4883_amd import workloads

    los, his = workloads.batch_intervals(0)
    n = len(los)
    nw = (his // 2 - los // 2 + 31) // 32
    offs = np.zeros(n, dtype=np.uint64)
    offs[1:] = np.cumsum(nw)[:-1]
    total = int(nw.sum())
    iv = np.zeros(n, dtype=sv.INTERVAL_DTYPE)
    iv["lo"], iv["hi"], iv["word_offset"], iv["flags"] = los, his, offs, 1
    words = torch.empty(total, dtype=torch.int32, device="cuda:0")
    stream = torch.cuda.current_stream(0)
    sv.sieve_set_timing(s.ctx, True)
    t_cold = time.perf_counter()
    pi = sv.sieve_batch(s.ctx, iv, words, total, stream=stream)  # cold: graph capture, prime table
    cold_ms = 1e3 * (time.perf_counter() - t_cold)
    tuning = None
    if tune:
        t_tune = time.perf_counter()
        best, best_ms = sv.sieve_autotune(s.ctx, iv, apply=True)
        tuning = {"chosen": best, "tuner_kernel_ms": best_ms,
                  "tune_s": time.perf_counter() - t_tune,
                  "note": "sieve_autotune on these 4096 intervals with their bitmaps; "
                          "candidates: the automatic plan, 4 segment sizes x 3 dense bounds, "
                          "then 1 or 2 workgroups per CU"}
        pi = sv.sieve_batch(s.ctx, iv, words, total, stream=stream)  # graph for the chosen tuning
    for _ in range(warmup):
        pi = sv.sieve_batch(s.ctx, iv, words, total, stream=stream)
    torch.cuda.synchronize()
    kms = []
    for _ in range(steps):  # graph time from HIP events around each launch
        pi = sv.sieve_batch(s.ctx, iv, words, total, stream=stream)
        kms.append(sv.sieve_last_kernel_ms(s.ctx))
    torch.cuda.synchronize()
    sv.sieve_set_timing(s.ctx, False)  # call time as in production use, no events
    t0 = time.perf_counter()
    for _ in range(steps):
        pi = sv.sieve_batch(s.ctx, iv, words, total, stream=stream)
    torch.cuda.synchronize()
    t_batch = (time.perf_counter() - t0) / steps
    ints = int((his - los).sum())
    rec = {"workload": "batched sieve: 4096 intervals [a, a+L), a log-uniform in [1e6, 1e12], "
                       "L log-uniform in [1e4, 1e8], seed 0; per-interval pi and packed bitmaps",
           "intervals": n, "integers": ints, "bitmap_bytes": 4 * total,
           "inputs_sha256": workloads.fingerprint(los, his),
           "ms_per_batch": 1e3 * t_batch, "graph_ms": float(np.mean(kms)), "cold_ms": cold_ms,
           "ints_per_s": ints / t_batch, "pi_sum": int(pi.sum()), "tuning": tuning}
    rec["_pi"] = pi
    # roofline of the batch graph (reset, batch kernel, reduction, counts
    # copy; the batch kernel dominates): the intervals' algorithmic LDS work
    # over the graph's event-timed duration
    primes = sv.sieve_base_primes(s.ctx, int(np.sqrt(float(his.max()))) + 2)
    g_ms = rec["graph_ms"]
    roof = measured_roofline(primes, zip(los.tolist(), his.tolist()), g_ms * 1e-3, peaks,
                             load_counters("batch-4096"), "batch-4096",
                             "batch graph (batch_kernel dominant)")
    roof["kernel_ms"] = g_ms
    rec["roofline"] = roof
    if check_plain:
        # the same outputs, one plain call per interval (pi returned per call),
        # kernel timing still off
        base = words.data_ptr()
        pis = np.zeros(n, dtype=np.uint64)
        sv.sieve_range_bitmap(s.ctx, int(los[0]), int(his[0]), base, int(nw[0]), True, stream=stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n):
            pis[i] = sv.sieve_range_bitmap(s.ctx, int(los[i]), int(his[i]), base + 4 * int(offs[i]),
                                           int(nw[i]), True, stream=stream)
        torch.cuda.synchronize()
        t_plain = time.perf_counter() - t0
        assert np.array_equal(pis, pi), "batched and plain counts differ"
        rec.update({"ms_plain_sequential": 1e3 * t_plain, "speedup_vs_plain": t_plain / t_batch})
    sv.sieve_set_timing(s.ctx, True)
    del words
    torch.cuda.empty_cache()
    return rec


def run_serve(sv, seconds, modes=("batched", "plain"), rate=2000.0):
    """Replay the served workload (Poisson arrivals, seed 1) for `seconds`
    through the native server in each mode; latency runs from each request's
    scheduled arrival to its result in host memory."""
    import numpy as np

    from paper_1205_4883_amd import workloads

    tr = workloads.serve_trace(1, seconds=seconds, rate=rate)
    flags = tr["bitmap"].astype(np.uint32)
    ints = int((tr["hi"] - tr["lo"]).sum())
    out = {"workload": f"served sieve: Poisson arrivals at {rate:g} req/s for {seconds:g} s (seed 1), "
                       "lo log-uniform in [1e3, 1e12], length log-uniform in [1e3, 1e9], "
                       "50% bitmap-return; 32 GiB HBM budget",
           "requests": int(tr["t"].size), "integers": ints,
           "bitmap_bytes": int(4 * ((tr["hi"] // 2 - tr["lo"] // 2 + 31) // 32)[tr["bitmap"]].sum()),
           "inputs_sha256": workloads.fingerprint(tr["lo"], tr["hi"])}
    pis, lats = {}, {}
    for mode in modes:
        m = sv.sieve.SIEVE_SERVE_PLAIN if mode == "plain" else sv.sieve.SIEVE_SERVE_BATCHED
        pi, lat, st = sv.sieve_serve_trace(0, tr["lo"], tr["hi"], flags, tr["t"], mode=m)
        span = float(np.max(tr["t"] + lat * 1e-3))
        out[mode] = {"p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
                     "span_s": span,
                     "mean_ms": float(lat.mean()), "max_ms": float(lat.max()),
                     "ints_per_s": ints / span, "batches": st["batches"],
                     "max_batch": st["max_batch_seen"], "max_inflight": st["max_inflight"],
                     "single_launches": st["single_launches"], "deferred": st["deferred"],
                     "graph_captures": st["graph_captures"], "device_pool_bytes": st["device_pool_bytes"],
                     "peak_admitted_bytes": st["peak_admitted_bytes"],
                     "max_launch_call_ms": st["max_launch_call_ns"] * 1e-6,
                     "slow_launch_calls": st["slow_launch_calls"]}
        pis[mode], lats[mode] = pi, lat
    if len(pis) == 2:
        assert np.array_equal(pis["batched"], pis["plain"]), "served results differ by mode"
        out["results_equal_across_modes"] = True
    # the slowest requests of the first mode, with what they asked for
    m0 = modes[0]
    slow = np.argsort(lats[m0])[-5:][::-1]
    out["slowest"] = [{"i": int(i), "t_s": float(tr["t"][i]), "lo": int(tr["lo"][i]),
                       "len": int(tr["hi"][i] - tr["lo"][i]), "bitmap": bool(tr["bitmap"][i]),
                       **{f"{m}_ms": float(lats[m][i]) for m in lats}} for i in slow]
    return out


def run_mr(sv, torch, steps, warmup, n=1 << 24):
    """Batched deterministic Miller-Rabin on n random odd 64-bit integers
    (seed 2), against the oracle's Miller-Rabin on the host."""
    import numpy as np

    import oracle  # CPU-baseline leg only

    rng = np.random.default_rng(2)
    ns = rng.integers(0, 2**63, n, dtype=np.uint64) * np.uint64(2) + np.uint64(1)
    s = sv.Sieve(0)
    sv.sieve_set_timing(s.ctx, True)
    d_n = torch.from_numpy(ns.view(np.int64)).to("cuda:0")
    out = torch.empty(n, dtype=torch.uint8, device="cuda:0")
    stream = torch.cuda.current_stream(0)
    for _ in range(warmup):
        sv.sieve_is_prime_batch(s.ctx, d_n, n, out, stream=stream)
    torch.cuda.synchronize()
    kms = []
    t0 = time.perf_counter()
    for _ in range(steps):
        sv.sieve_is_prime_batch(s.ctx, d_n, n, out, stream=stream)
        kms.append(sv.sieve_last_kernel_ms(s.ctx))
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / steps
    got = out.cpu().numpy()
    s.close()
    sample = 1 << 16
    t1 = time.perf_counter()
    want = np.array([oracle.mr_is_prime(int(x)) for x in ns[:sample]], dtype=np.uint8)
    cpu_dt = time.perf_counter() - t1
    assert np.array_equal(got[:sample], want), "GPU and oracle Miller-Rabin differ"
    return {"workload": f"deterministic Miller-Rabin of {n} random odd 64-bit integers (seed 2)",
            "candidates": n, "primes": int(got.sum()), "ms_per_batch": 1e3 * dt,
            "kernel_ms": float(np.mean(kms)), "candidates_per_s": n / dt,
            "cpu_baseline": {"value": sample / cpu_dt, "unit": "candidates/s", "cores": 1,
                             "kind": "oracle", "sample": f"first {sample} candidates, one thread, "
                                                         "called one by one from Python"}}


def cpu_baseline(lo, hi, expect_pi, bitmap=False):
    """The oracle on the whole range on every host thread, and on one thread
    over the range's last tenth (its densest part): the count, or with bitmap
    the packed words and the count, as the GPU leg produces them."""
    import oracle  # CPU-baseline leg only

    oracle.build(force=False)
    threads = oracle.default_threads()
    run = (lambda a, b, t: oracle.bitmap(a, b, threads=t)[1]) if bitmap else \
          (lambda a, b, t: oracle.count(a, b, threads=t))
    what = "bitmap and count" if bitmap else "count"
    t0 = time.perf_counter()
    pi = run(lo, hi, threads)
    dt = time.perf_counter() - t0
    assert pi == expect_pi, (pi, expect_pi)
    lo1 = hi - (hi - lo) // 10
    t1 = time.perf_counter()
    run(lo1, hi, 1)
    dt1 = time.perf_counter() - t1
    return {"value": (hi - lo) / dt, "unit": "ints/s", "cores": threads, "kind": "oracle",
            "sample": f"the whole workload: oracle {what} of [{lo}, {hi}) on {threads} threads, "
                      f"{dt:.2f} s, pi={pi}",
            "one_thread": {"value": (hi - lo1) / dt1, "unit": "ints/s", "cores": 1,
                           "sample": f"oracle {what} of [{lo1}, {hi}) on one thread, {dt1:.2f} s"},
            "host": host_info(threads)}


def batch_cpu_baseline(sv, pi_gpu, n_sample=512):
    """The oracle's counts of the first n_sample batch intervals on every host
    thread (one interval at a time), checked against the batch's counts."""
    import numpy as np

    import oracle  # CPU-baseline leg only

    from paper_1205_4883_amd import workloads

    oracle.build(force=False)
    threads = oracle.default_threads()
    los, his = workloads.batch_intervals(0)
    los, his = los[:n_sample].tolist(), his[:n_sample].tolist()
    t0 = time.perf_counter()
    pis = [oracle.count(a, b, threads=threads) for a, b in zip(los, his)]
    dt = time.perf_counter() - t0
    assert np.array_equal(np.array(pis, dtype=np.uint64), np.asarray(pi_gpu[:n_sample])), \
        "oracle and batch counts differ"
    ints = sum(b - a for a, b in zip(los, his))
    return {"value": ints / dt, "unit": "ints/s", "cores": threads, "kind": "oracle",
            "sample": f"counts of the first {n_sample} of the 4096 intervals ({ints} integers), "
                      f"one interval at a time on {threads} threads, {dt:.2f} s; equal to the "
                      "batch's counts",
            "host": host_info(threads)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    # enough warm-up for the shader clock to leave its idle level (a cold
    # [2, 1e10) kernel runs about 6% slower over its first ten launches)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=50)
    ap.add_argument("--workload", default="count-1e10",
                    choices=sorted(WORKLOADS) + ["batch-4096", "serve-2000", "mr-2e24"])
    ap.add_argument("--serve-seconds", type=float, default=None,
                    help="trace length for the served workload (serve-2000: 60, default line: 5)")
    ap.add_argument("--serve-rates", default="20000,100000",
                    help="serve-2000 only: extra arrival rates (req/s) replayed for 2 s each, both modes")
    ap.add_argument("--no-batch", action="store_true",
                    help="skip the batch, serving and Miller-Rabin blocks of the default line")
    ap.add_argument("--no-cpu", action="store_true", help="skip the CPU oracle baseline")
    ap.add_argument("--no-plain", action="store_true",
                    help="batch-4096: skip the 4096 one-at-a-time calls (e.g. under a profiler)")
    ap.add_argument("--seg-bits", type=int, default=0, help="tuning: odd integers per segment")
    ap.add_argument("--dense-limit", type=int, default=0, help="tuning: wave-per-prime bound")
    ap.add_argument("--block-threads", type=int, default=0, help="tuning: threads per workgroup")
    ap.add_argument("--bucket-limit", type=int, default=0,
                    help="tuning: primes from here on go through hit buckets (0 automatic, 4294967295 never)")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the LDS and VALU microbenchmarks (sieve_measure_peaks) and print them")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB three times (the "
                         "reference kernel for scaling rocprofv3 FETCH_SIZE/WRITE_SIZE)")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU "
              "split of a range (shards of ceil(n/G) integers, one 8-byte sum) is designed but not "
              "built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    if args.calibrate_copy:
        n = args.calibrate_copy * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.int32, device="cuda:0")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": 4 * n, "copies": 3}), flush=True)
        return

    import paper_1205_4883_amd as sv

    if args.peaks:
        s = sv.Sieve(0)
        print(json.dumps({"peaks": sv.sieve_measure_peaks(s.ctx)}), flush=True)
        s.close()
        return

    if args.workload == "mr-2e24":
        r = run_mr(sv, torch, args.steps, args.warmup)
        print(json.dumps({
            "metric": "Miller-Rabin candidates/s (64-bit)", "value": r["candidates_per_s"],
            "unit": "candidates/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": r["ms_per_batch"], "higher_is_better": True, "scaling": "weak",
            "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": r["workload"]}, "mr": r}), flush=True)
        return

    if args.workload == "serve-2000":
        secs = args.serve_seconds or 60.0
        r = run_serve(sv, secs)
        r["load_sweep"] = [run_serve(sv, 2.0, rate=float(x)) for x in args.serve_rates.split(",") if x]
        print(json.dumps({
            "metric": METRIC, "value": r["batched"]["ints_per_s"], "unit": "ints/s", "n_gpus": 1,
            "steps": 1, "warmup": 0, "ms_per_step": 1e3 * secs, "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "u64", "data": "synthetic",
            "config": {"workload": r["workload"]}, "serve": r}), flush=True)
        return

    s = sv.Sieve(0)
    peaks = sv.sieve_measure_peaks(s.ctx)  # this device's LDS and VALU rates, measured
    if args.seg_bits or args.dense_limit or args.block_threads or args.bucket_limit:
        s.tuning(seg_bits=args.seg_bits, dense_limit=args.dense_limit, block_threads=args.block_threads,
                 bucket_limit=args.bucket_limit)

    if args.workload == "batch-4096":
        b = run_batch(sv, torch, s, args.steps, args.warmup, check_plain=not args.no_plain,
                      tune=not (args.seg_bits or args.dense_limit or args.block_threads), peaks=peaks)
        s.close()
        pi = b.pop("_pi")
        if not args.no_cpu:
            b["cpu_baseline"] = batch_cpu_baseline(sv, pi)
        print(json.dumps({
            "metric": METRIC, "value": b["ints_per_s"], "unit": "ints/s", "n_gpus": 1,
            "steps": args.steps, "warmup": args.warmup, "ms_per_step": b["ms_per_batch"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u64",
            "data": "synthetic", "config": {"workload": b["workload"]}, "peaks": peaks,
            "batch": b}), flush=True)
        return

    wl = WORKLOADS[args.workload]
    lo, hi = wl["lo"], wl["hi"]
    r = run_single(sv, torch, s, wl, args.steps, args.warmup, peaks, args.workload,
                   latency_calls=1000 if args.workload == "bitmap-1e7" else 0)
    device = device_info(torch)
    plan = r["plan"]
    rec = {
        "metric": METRIC,
        "value": r["ints_per_s"],
        "unit": "ints/s",
        "n_gpus": 1,
        "steps": r["calls"],
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_call"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        # u64 segment bases and offsets above 2^32, 32-bit words and marks
        "dtype": "u64" if hi > 1 << 32 else "u32",
        "data": "synthetic",
        "cold_ms": r["cold_ms"],
        "call_ms": r["call_ms"],
        "device": device,
        "config": {"workload": wl["name"], "lo": lo, "hi": hi, "pi": r["pi"],
                   "presieve_primes": PRESIEVE_PRIMES, **plan},
        "roofline": r["roofline"],
        "peaks": peaks,
    }
    if args.workload == "count-1e10" and not args.no_batch:
        # the other configurations, each in a block of its own
        for key in ("bitmap-1e7", "bitmap-1e9"):
            w = WORKLOADS[key]
            rec["c1" if key == "bitmap-1e7" else "c2"] = run_single(
                sv, torch, s, w, 200 if key == "bitmap-1e9" else 100, 50, peaks, key,
                latency_calls=1000 if key == "bitmap-1e7" else 0)
        rec["batch"] = run_batch(sv, torch, s, steps=20, warmup=5, peaks=peaks)
    s.close()
    if args.workload == "count-1e10" and not args.no_batch:
        rec["serve"] = run_serve(sv, args.serve_seconds or 60.0)
        rec["serve"]["load_sweep"] = [run_serve(sv, 2.0, rate=20000.0)]
        rec["mr"] = run_mr(sv, torch, steps=20, warmup=5)
    if not args.no_cpu:
        rec["cpu_baseline"] = cpu_baseline(lo, hi, wl["pi"], bitmap=wl["bitmap"])
        if "batch" in rec:
            rec["batch"]["cpu_baseline"] = batch_cpu_baseline(sv, rec["batch"]["_pi"])
    if "batch" in rec:
        rec["batch"].pop("_pi")
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
