// Microbenchmarks of the two units the segment kernels load: LDS 32-bit
// atomic ORs (the crossing-off of Section 3.1) and int32 VALU issue.  Each
// kernel runs a fixed, bounded amount of work on every CU and exits; the
// host times it with HIP events.  Every workgroup also samples the shader
// cycle counter and the constant-rate wall counter at its start and end, so
// the clock the kernels actually ran at is measured, not assumed.
#include <algorithm>
#include <vector>

#include "sieve_runtime.h"

namespace {

constexpr uint32_t kThreads = 1024;   // 16 wavefronts, as the segment kernels
constexpr uint32_t kWordsPerWave = 64;
constexpr uint32_t kLdsUnroll = 16;   // atomics in flight per lane per pass
constexpr uint32_t kValuUnroll = 64;  // VALU instructions per lane per pass

struct ClockSample {
    unsigned long long t0, t1, w0, w1;  // cycle counter, wall counter
};

__device__ __forceinline__ void sample_start(ClockSample *cs)
{
    if (threadIdx.x == 0) {
        cs[blockIdx.x].t0 = clock64();
        cs[blockIdx.x].w0 = wall_clock64();
    }
}

__device__ __forceinline__ void sample_end(ClockSample *cs)
{
    if (threadIdx.x == 0) {
        cs[blockIdx.x].t1 = clock64();
        cs[blockIdx.x].w1 = wall_clock64();
    }
}

// mode 0: ds_or_b32, lane l of each half-wavefront on bank l (32 distinct
//         banks: conflict-free);
// mode 1: ds_write_b32, same addresses;
// mode 2: ds_or_b32 at random words of a 16,384-word array (the pattern of
//         one-lane-per-prime marking): each lane cycles through 16 hashed
//         words, so the banks of a half-wavefront are independent and
//         uniform;
// mode 3: ds_read_b32, same addresses as mode 0 (summed into a register);
// mode 4: ds_write_b64, lane l of each half-wavefront on banks 2l, 2l + 1;
// mode 5: mode 0 with only the even lanes active (half the lanes masked off).
template <int kMode>
__global__ void __launch_bounds__(kThreads) lds_peak_kernel(uint32_t passes, ClockSample *cs, uint32_t *sink)
{
    constexpr uint32_t kWords = kMode == 2 ? 16384u : (kMode == 4 ? 2 : 1) * (kThreads / 64) * kWordsPerWave;
    __shared__ __align__(16) uint32_t lds[kWords];
    for (uint32_t i = threadIdx.x; i < kWords; i += blockDim.x)
        lds[i] = 0;
    __syncthreads();
    sample_start(cs);
    const uint32_t lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    uint32_t addr = wave * kWordsPerWave + lane;
    // mode 2: kLdsUnroll random words per lane, hashed once and kept in
    // registers, so that the loop issues nothing but the atomics
    uint32_t rnd[kLdsUnroll];
#pragma unroll
    for (uint32_t k = 0; k < kLdsUnroll; ++k) {
        uint32_t h = (threadIdx.x * kLdsUnroll + k) * 2654435761u + blockIdx.x * 40503u;
        h ^= h >> 16;
        h *= 0x7feb352du;
        h ^= h >> 15;
        h *= 0x846ca68bu;
        h ^= h >> 16;
        rnd[k] = h & 16383u;
    }
    uint32_t acc = 0;
    const bool active = kMode != 5 || (lane & 1) == 0;
    for (uint32_t p = 0; active && p < passes; ++p) {
#pragma unroll
        for (uint32_t k = 0; k < kLdsUnroll; ++k) {
            if (kMode == 2)
                addr = rnd[k];
            const uint32_t bit = 1u << ((threadIdx.x + k) & 31);  // per-lane constants: no VALU in the loop
            if (kMode == 1) {
                __hip_atomic_store(&lds[addr], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if (kMode == 3) {
                acc += __hip_atomic_load(&lds[(addr + k) & (kWords - 1)], __ATOMIC_RELAXED,
                                         __HIP_MEMORY_SCOPE_WORKGROUP);
            } else if (kMode == 4) {
                auto *w2 = reinterpret_cast<unsigned long long *>(lds);
                __hip_atomic_store(&w2[(wave * kWordsPerWave + lane + 64 * (k & 1)) & (kWords / 2 - 1)],
                                   (static_cast<unsigned long long>(k) << 32) | bit, __ATOMIC_RELAXED,
                                   __HIP_MEMORY_SCOPE_WORKGROUP);
            } else {
                __hip_atomic_fetch_or(&lds[addr], bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
            }
        }
    }
    __syncthreads();
    sample_end(cs);
    if (threadIdx.x == 0)
        sink[blockIdx.x] = lds[0] + acc;  // keeps the stores and loads live
    else if (acc == 0x12345678u)
        sink[blockIdx.x] = acc;
}

// Four independent dependency chains of v_add_u32 / v_xor_b32, written as
// inline VALU instructions (no memory operands), so that the count per pass
// is exact: kValuUnroll instructions per lane per pass.
__global__ void __launch_bounds__(kThreads) valu_peak_kernel(uint32_t passes, ClockSample *cs, uint32_t *sink)
{
    sample_start(cs);
    uint32_t a = threadIdx.x, b = blockIdx.x, c = a ^ 0x9e3779b9u, d = b + 0x7f4a7c15u;
    const uint32_t k1 = 0x85ebca6bu, k2 = 0xc2b2ae35u;
    for (uint32_t p = 0; p < passes; ++p) {
#pragma unroll
        for (uint32_t k = 0; k < kValuUnroll / 8; ++k) {
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(a) : "v"(k1));
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(b) : "v"(k2));
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(c) : "v"(k1));
            asm volatile("v_add_u32 %0, %0, %1" : "+v"(d) : "v"(k2));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(a) : "v"(k2));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(b) : "v"(k1));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(c) : "v"(k2));
            asm volatile("v_xor_b32 %0, %0, %1" : "+v"(d) : "v"(k1));
        }
    }
    sample_end(cs);
    const uint32_t v = a ^ b ^ c ^ d;
    if (v == 0x12345678u)  // practically never: keeps the chains live
        sink[blockIdx.x] = v;
}

// Shader clock over the launch: cycles / wall time, averaged over the
// workgroups (wall counter at wall_hz).
double clock_hz(const std::vector<ClockSample> &cs, double wall_hz)
{
    double cyc = 0, wall = 0;
    for (const ClockSample &s : cs) {
        cyc += static_cast<double>(s.t1 - s.t0);
        wall += static_cast<double>(s.w1 - s.w0);
    }
    return wall > 0 ? cyc / wall * wall_hz : 0;
}

}  // namespace

extern "C" {

int sieve_measure_peaks(sieve_ctx *c, sieve_peaks *out)
{
    if (!c || !out)
        return SIEVE_EINVAL;
    SV_HIP_TRY(c, hipSetDevice(c->device));
    int wall_khz = 0;
    SV_HIP_TRY(c, hipDeviceGetAttribute(&wall_khz, hipDeviceAttributeWallClockRate, c->device));
    const uint32_t grid = 4 * c->n_cu;  // two rounds of two 1024-thread workgroups per CU
    ClockSample *d_cs = nullptr;
    uint32_t *d_sink = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    int st = SIEVE_OK;
    sieve_peaks r{};
    r.n_cu = c->n_cu;
    std::vector<ClockSample> cs(grid);
    auto fail = [&](hipError_t e) {
        c->last_hip = e;
        st = SIEVE_EDEVICE;
    };
    // time one launch (after one warm-up launch); returns ms, fills cs
    auto run = [&](auto launch) -> double {
        float ms = 0;
        hipError_t e = hipSuccess;
        for (int rep = 0; rep < 2 && e == hipSuccess; ++rep) {
            if ((e = hipEventRecord(e0, c->stream)) != hipSuccess)
                break;
            launch();
            if ((e = hipGetLastError()) != hipSuccess || (e = hipEventRecord(e1, c->stream)) != hipSuccess ||
                (e = hipEventSynchronize(e1)) != hipSuccess || (e = hipEventElapsedTime(&ms, e0, e1)) != hipSuccess)
                break;
        }
        if (e == hipSuccess)
            e = hipMemcpy(cs.data(), d_cs, grid * sizeof(ClockSample), hipMemcpyDeviceToHost);
        if (e != hipSuccess) {
            fail(e);
            return 0;
        }
        return ms;
    };
    do {
        hipError_t e;
        if ((e = hipMalloc(&d_cs, grid * sizeof(ClockSample))) != hipSuccess ||
            (e = hipMalloc(&d_sink, grid * sizeof(uint32_t))) != hipSuccess ||
            (e = hipEventCreate(&e0)) != hipSuccess || (e = hipEventCreate(&e1)) != hipSuccess) {
            fail(e);
            break;
        }
        const double wall_hz = 1e3 * wall_khz;
        const double lanes = static_cast<double>(grid) * kThreads;
        const uint32_t lds_passes = 4096, valu_passes = 2048;
        double ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<0>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.lds_or_lane_ops_per_s = lanes * lds_passes * kLdsUnroll / (ms * 1e-3);
        r.lds_or_clock_hz = clock_hz(cs, wall_hz);
        ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<1>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.lds_write_lane_ops_per_s = lanes * lds_passes * kLdsUnroll / (ms * 1e-3);
        ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<2>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes / 4, d_cs,
                               d_sink);
        });
        if (st)
            break;
        r.lds_or_scatter_lane_ops_per_s = lanes * (lds_passes / 4) * kLdsUnroll / (ms * 1e-3);
        ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<3>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.lds_read_lane_ops_per_s = lanes * lds_passes * kLdsUnroll / (ms * 1e-3);
        ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<4>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.lds_write_b64_bytes_per_s = 8 * lanes * lds_passes * kLdsUnroll / (ms * 1e-3);
        ms = run([&] {
            hipLaunchKernelGGL(lds_peak_kernel<5>, dim3(grid), dim3(kThreads), 0, c->stream, lds_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.lds_or_half_lanes_wave_instr_per_s = (lanes / 64) * lds_passes * kLdsUnroll / (ms * 1e-3);
        r.lds_or_wave_instr_per_s = r.lds_or_lane_ops_per_s / 64;
        ms = run([&] {
            hipLaunchKernelGGL(valu_peak_kernel, dim3(grid), dim3(kThreads), 0, c->stream, valu_passes, d_cs, d_sink);
        });
        if (st)
            break;
        r.valu_wave_instr_per_s = static_cast<double>(grid) * (kThreads / 64) * valu_passes * kValuUnroll / (ms * 1e-3);
        r.valu_clock_hz = clock_hz(cs, wall_hz);
        const double clk = r.valu_clock_hz > 0 ? r.valu_clock_hz : 2.4e9;
        r.valu_wave_instr_per_clk_cu = r.valu_wave_instr_per_s / (clk * c->n_cu);
        const double lclk = r.lds_or_clock_hz > 0 ? r.lds_or_clock_hz : 2.4e9;
        r.lds_or_lanes_per_clk_cu = r.lds_or_lane_ops_per_s / (lclk * c->n_cu);
    } while (false);
    if (d_cs)
        (void)hipFree(d_cs);
    if (d_sink)
        (void)hipFree(d_sink);
    if (e0)
        (void)hipEventDestroy(e0);
    if (e1)
        (void)hipEventDestroy(e1);
    if (st == SIEVE_OK)
        *out = r;
    return st;
}

}  // extern "C"
