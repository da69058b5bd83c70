// Random-gather rates of the device, the roofline the walkers are compared
// against: walker steps are chains of dependent 4-8 byte loads at random
// addresses, so neither streaming bandwidth nor MFMA rate bounds them.
//
//   independent: every lane issues `in_flight` independent random 8-byte loads
//                per round (addresses from a hash of lane and round), so the
//                memory system sees up to lanes x in_flight requests at once;
//   chase:       every lane follows its own pointer chain through a random
//                cyclic order of 64-byte lines (one dependent load per hop),
//                the access pattern of a walker;
//   mixed:       as independent, plus one random 8-byte store per round, so
//                one store for every `in_flight` loads (the walkers also
//                write their state words at random places); a store reaches
//                memory as a partial (32-byte) write;
//   mixed lines: as mixed, but the store fills a whole random 64-byte line
//                (a full-line write, as the evictions of lines the walkers
//                have written throughout);
//   lds:         every lane issues `in_flight` independent random 4-byte
//                reads per round from a 64 KiB table in its workgroup's LDS,
//                each round's addresses depending on the previous round's
//                values (the working set is fixed: the LDS random-access rate).
// All report memory operations (loads, and stores in mixed mode) per second
// over a working set of the given size, which
// selects the cache tier (L2 4 MB per XCD, 256 MB Infinity Cache, HBM).  A
// sweep over lanes (and loads in flight) gives the peak of each tier.
//
// flavor selects how the loads are issued: 0 plain loads, 1 non-temporal
// loads, 2 relaxed atomic loads at device scope, 3 relaxed atomic loads at
// system scope (the cache policy bits differ; the rate and the bytes each
// load fetches from memory show which suits scattered 8-byte words).
#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lap_launch.h"
#include "../../include/lap.h"

namespace lap {

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

template <int F>
__device__ __forceinline__ uint64_t load_word(const uint64_t *p) {
    if constexpr (F == 1) {
        return __builtin_nontemporal_load(p);
    } else if constexpr (F == 2) {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    } else if constexpr (F == 3) {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    } else {
        return *p;
    }
}

// line i (8 words) holds in word 0 the index of the next line of the chain:
// next = (a * i + c) mod n_lines with n_lines a power of two, a = 5 mod 8,
// c odd: a full-period permutation.
__global__ void chase_init_kernel(uint64_t *buf, uint64_t n_lines, uint64_t a, uint64_t c) {
    const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
    for (uint64_t i = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n_lines; i += stride)
        buf[i * 8] = (a * i + c) & (n_lines - 1);
}

template <int F>
__global__ __launch_bounds__(256) void chase_kernel(const uint64_t *buf, uint64_t n_lines, int64_t hops,
                                                    uint64_t *sink) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t p = mix64(gid) & (n_lines - 1);
    for (int64_t h = 0; h < hops; ++h) p = load_word<F>(buf + p * 8) & (n_lines - 1);
    if (p == 0xFFFFFFFFFFFFFFFFull) sink[0] = p;
}

template <int D, int F>
__global__ __launch_bounds__(256) void gather_kernel(const uint64_t *buf, uint64_t n_words, int64_t rounds,
                                                     uint64_t *sink) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint64_t acc = 0;
    for (int64_t r = 0; r < rounds; ++r) {
        uint64_t v[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            v[j] = load_word<F>(buf + (mix64(gid * 0x9E3779B97F4A7C15ull + (uint64_t)r * D + j) & (n_words - 1)));
#pragma unroll
        for (int j = 0; j < D; ++j) acc ^= v[j];
    }
    if (acc == 0x1234567) sink[0] = acc;
}

// each round: D random loads, then one random store of their combination to a
// third random word (its address from another hash of lane and round)
// (LINE: the store covers the whole 64-byte line of that word)
template <int D, bool LINE>
__global__ __launch_bounds__(256) void mixed_kernel(uint64_t *buf, uint64_t n_words, int64_t rounds) {
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    for (int64_t r = 0; r < rounds; ++r) {
        uint64_t v[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            v[j] = buf[mix64(gid * 0x9E3779B97F4A7C15ull + (uint64_t)r * D + j) & (n_words - 1)];
        uint64_t acc = 0;
#pragma unroll
        for (int j = 0; j < D; ++j) acc ^= v[j];
        const uint64_t at = mix64(~(gid * 0xD1B54A32D192ED03ull) + (uint64_t)r) & (n_words - 1);
        if constexpr (LINE) {
            uint64_t *line = buf + (at & ~7ull);
#pragma unroll
            for (int j = 0; j < 8; ++j) line[j] = acc + (uint64_t)j;
        } else {
            buf[at] = acc | 1ull;
        }
    }
}

template <bool LINE>
void launch_mixed(int depth, unsigned grid, hipStream_t s, uint64_t *buf, uint64_t words, int64_t rounds) {
    switch (depth) {
        case 1: hipLaunchKernelGGL((mixed_kernel<1, LINE>), dim3(grid), dim3(256), 0, s, buf, words, rounds); break;
        case 2: hipLaunchKernelGGL((mixed_kernel<2, LINE>), dim3(grid), dim3(256), 0, s, buf, words, rounds); break;
        case 4: hipLaunchKernelGGL((mixed_kernel<4, LINE>), dim3(grid), dim3(256), 0, s, buf, words, rounds); break;
        case 8: hipLaunchKernelGGL((mixed_kernel<8, LINE>), dim3(grid), dim3(256), 0, s, buf, words, rounds); break;
        default: hipLaunchKernelGGL((mixed_kernel<16, LINE>), dim3(grid), dim3(256), 0, s, buf, words, rounds); break;
    }
}

template <int D>
__global__ __launch_bounds__(256) void lds_kernel(int64_t rounds, uint64_t *sink) {
    constexpr int kWords = 16384;   // 64 KiB
    __shared__ uint32_t tab[kWords];
    for (int i = (int)threadIdx.x; i < kWords; i += (int)blockDim.x) tab[i] = (uint32_t)mix64((uint64_t)i);
    __syncthreads();
    const uint64_t gid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t acc = 0;
    for (int64_t r = 0; r < rounds; ++r) {
        uint32_t v[D];
#pragma unroll
        for (int j = 0; j < D; ++j)
            v[j] = tab[(uint32_t)mix64(gid * 0x9E3779B97F4A7C15ull + (uint64_t)r * D + j + acc) & (kWords - 1)];
#pragma unroll
        for (int j = 0; j < D; ++j) acc ^= v[j];
    }
    if (acc == 0x1234567u) sink[0] = acc;
}

void launch_lds(int depth, unsigned grid, hipStream_t s, int64_t rounds, uint64_t *sink) {
    switch (depth) {
        case 1: hipLaunchKernelGGL(lds_kernel<1>, dim3(grid), dim3(256), 0, s, rounds, sink); break;
        case 2: hipLaunchKernelGGL(lds_kernel<2>, dim3(grid), dim3(256), 0, s, rounds, sink); break;
        case 4: hipLaunchKernelGGL(lds_kernel<4>, dim3(grid), dim3(256), 0, s, rounds, sink); break;
        case 8: hipLaunchKernelGGL(lds_kernel<8>, dim3(grid), dim3(256), 0, s, rounds, sink); break;
        default: hipLaunchKernelGGL(lds_kernel<16>, dim3(grid), dim3(256), 0, s, rounds, sink); break;
    }
}

template <int F>
void launch_gather_depth(int depth, unsigned grid, hipStream_t s, const uint64_t *buf, uint64_t words,
                         int64_t rounds, uint64_t *sink) {
    switch (depth) {
        case 1: hipLaunchKernelGGL((gather_kernel<1, F>), dim3(grid), dim3(256), 0, s, buf, words, rounds, sink); break;
        case 2: hipLaunchKernelGGL((gather_kernel<2, F>), dim3(grid), dim3(256), 0, s, buf, words, rounds, sink); break;
        case 4: hipLaunchKernelGGL((gather_kernel<4, F>), dim3(grid), dim3(256), 0, s, buf, words, rounds, sink); break;
        case 8: hipLaunchKernelGGL((gather_kernel<8, F>), dim3(grid), dim3(256), 0, s, buf, words, rounds, sink); break;
        default: hipLaunchKernelGGL((gather_kernel<16, F>), dim3(grid), dim3(256), 0, s, buf, words, rounds, sink); break;
    }
}

void launch_gather(int flavor, int depth, unsigned grid, hipStream_t s, const uint64_t *buf, uint64_t words,
                   int64_t rounds, uint64_t *sink) {
    switch (flavor) {
        case 1: launch_gather_depth<1>(depth, grid, s, buf, words, rounds, sink); break;
        case 2: launch_gather_depth<2>(depth, grid, s, buf, words, rounds, sink); break;
        case 3: launch_gather_depth<3>(depth, grid, s, buf, words, rounds, sink); break;
        default: launch_gather_depth<0>(depth, grid, s, buf, words, rounds, sink); break;
    }
}

void launch_chase(int flavor, unsigned grid, hipStream_t s, const uint64_t *buf, uint64_t n_lines, int64_t hops,
                  uint64_t *sink) {
    switch (flavor) {
        case 1: hipLaunchKernelGGL(chase_kernel<1>, dim3(grid), dim3(256), 0, s, buf, n_lines, hops, sink); break;
        case 2: hipLaunchKernelGGL(chase_kernel<2>, dim3(grid), dim3(256), 0, s, buf, n_lines, hops, sink); break;
        case 3: hipLaunchKernelGGL(chase_kernel<3>, dim3(grid), dim3(256), 0, s, buf, n_lines, hops, sink); break;
        default: hipLaunchKernelGGL(chase_kernel<0>, dim3(grid), dim3(256), 0, s, buf, n_lines, hops, sink); break;
    }
}

}  // namespace lap

using namespace lap;

extern "C" int lap_bench_gather(int64_t bytes, int64_t lanes, int32_t mode, int32_t in_flight, int32_t flavor,
                                double *rate, void *hip_stream) {
    if (bytes < (1 << 20) || lanes < 256 || lanes > ((int64_t)1 << 24) || !rate || mode < 0 || mode > 4 ||
        (mode >= 2 && flavor != 0) ||
        (in_flight != 1 && in_flight != 2 && in_flight != 4 && in_flight != 8 && in_flight != 16) || flavor < 0 ||
        flavor > 3)
        return LAP_EINVAL;
    uint64_t words = 1;
    while (words * 2 * 8 <= (uint64_t)bytes) words *= 2;
    hipStream_t s = (hipStream_t)hip_stream;
    uint64_t *buf = nullptr, *sink = nullptr;
    if (hipMalloc(&buf, words * 8) != hipSuccess) return LAP_ENOMEM;
    if (hipMalloc(&sink, 64) != hipSuccess) {
        (void)hipFree(buf);
        return LAP_ENOMEM;
    }
    const uint64_t n_lines = words / 8;
    int rc = LAP_OK;
    hipLaunchKernelGGL(chase_init_kernel, dim3(4096), dim3(256), 0, s, buf, n_lines, 0x5DEECE66Dull * 8 + 5,
                       0x2545F4914F6CDD1Dull | 1ull);
    const unsigned grid = (unsigned)((lanes + 255) / 256);
    // work per lane: rounds of in_flight loads, or hops, about 512 loads either way
    const int64_t work = mode == 1 ? 512 : 512 / in_flight;
    hipEvent_t a, b;
    (void)hipEventCreate(&a);
    (void)hipEventCreate(&b);
    for (int rep = 0; rep < 2; ++rep) {           // first pass warms the caches
        (void)hipEventRecord(a, s);
        if (mode == 0)
            launch_gather(flavor, in_flight, grid, s, buf, words, work, sink);
        else if (mode == 1)
            launch_chase(flavor, grid, s, buf, n_lines, work, sink);
        else if (mode == 2)
            launch_mixed<false>(in_flight, grid, s, buf, words, work);
        else if (mode == 3)
            launch_mixed<true>(in_flight, grid, s, buf, words, work);
        else
            launch_lds(in_flight, grid, s, work * 4, sink);
        (void)hipEventRecord(b, s);
    }
    if (hipGetLastError() != hipSuccess || hipEventSynchronize(b) != hipSuccess) rc = LAP_EDEVICE;
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, a, b);
    // loads and stores per round (a line store counts once: one write request)
    const double per_round = mode == 0 ? (double)in_flight : mode == 1 ? 1.0
                           : mode == 4 ? 4.0 * (double)in_flight : (double)in_flight + 1.0;
    const double ops = (double)grid * 256.0 * (double)work * per_round;
    *rate = ms > 0 ? ops / (ms * 1e-3) : 0.0;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    (void)hipFree(buf);
    (void)hipFree(sink);
    return rc;
}
