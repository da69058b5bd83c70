// Device-side building blocks shared by the library's kernels: Philox draws,
// the neighbour-index map, packed per-node walk state and kernel parameters.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lap {

// ---------------------------------------------------------------- Philox4x64-10
// Counter-based generator of Salmon, Moraes, Dror and Shaw (SC'11): ten rounds
// of two 64x64->128 multiplies with the published multipliers and Weyl key
// increments.  Only word 0 of the output block is used.
__device__ __forceinline__ uint64_t philox_w0(uint64_t c0, uint64_t c1, uint64_t c2, uint64_t c3,
                                              uint64_t k0, uint64_t k1) {
    constexpr uint64_t kMulA = 0xD2E7470EE14C6C93ull;
    constexpr uint64_t kMulB = 0xCA5A826395121157ull;
    constexpr uint64_t kWeylA = 0x9E3779B97F4A7C15ull;
    constexpr uint64_t kWeylB = 0xBB67AE8584CAA73Bull;
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t pa_lo = kMulA * c0, pa_hi = __umul64hi(kMulA, c0);
        const uint64_t pb_lo = kMulB * c2, pb_hi = __umul64hi(kMulB, c2);
        const uint64_t n0 = pb_hi ^ c1 ^ k0;
        const uint64_t n2 = pa_hi ^ c3 ^ k1;
        c0 = n0;
        c1 = pb_lo;
        c2 = n2;
        c3 = pa_lo;
        k0 += kWeylA;
        k1 += kWeylB;
    }
    return c0;
}

// index in [0, d) for a 64-bit draw: the high word of x * d
__device__ __forceinline__ uint64_t pick_below(uint64_t x, uint64_t d) { return __umul64hi(x, d); }

// ------------------------------------------------------------ adjacency records
// nbr[u] packs the row offset (low 40 bits) and the degree (high 24 bits) so a
// walker gets both with one 8-byte load.
__device__ __forceinline__ int64_t nbr_off(uint64_t r) { return (int64_t)(r & ((1ull << 40) - 1)); }
__device__ __forceinline__ uint32_t nbr_deg(uint64_t r) { return (uint32_t)(r >> 40); }

// ------------------------------------------------------------ per-node walk state
// One 64-bit word per node per sample slot:
//   bits  0..31  next   (last draw at the node: its stack top)
//   bits 32..52  k      (draws made at the node in this sample)
//   bits 53..62  tag    (0 free, 1..512 on the path of walker tag-1 of the
//                        sample's wave or workgroup, 1023 in tree)
//   bit  63      epoch  (parity of the slot's sample counter; a word from the
//                        previous sample reads as free with k = 0)
constexpr uint32_t kTagFree = 0;
constexpr uint32_t kTagTree = 1023;
constexpr uint32_t kMaxWalkers = 512;
constexpr uint32_t kMaxDraws = (1u << 21) - 1;

__device__ __forceinline__ uint64_t st_pack(int32_t nxt, uint32_t k, uint32_t tag, uint32_t ep) {
    return (uint64_t)(uint32_t)nxt | ((uint64_t)k << 32) | ((uint64_t)tag << 53) |
           ((uint64_t)ep << 63);
}
__device__ __forceinline__ bool st_current(uint64_t w, uint32_t ep) { return (uint32_t)(w >> 63) == ep; }
__device__ __forceinline__ int32_t st_next(uint64_t w) { return (int32_t)(uint32_t)w; }
__device__ __forceinline__ uint32_t st_k(uint64_t w, uint32_t ep) {
    return st_current(w, ep) ? (uint32_t)((w >> 32) & 0x1FFFFFu) : 0u;
}
__device__ __forceinline__ uint32_t st_tag(uint64_t w, uint32_t ep) {
    return st_current(w, ep) ? (uint32_t)((w >> 53) & 0x3FFu) : kTagFree;
}

// ------------------------------------------------------------ LDS lane form
// The LDS-resident lane form keeps the CSR and one 32-bit word per node for
// each of its lanes' samples in LDS:
//   bits  0..9   next (graphs of at most kLdsMaxNodes nodes)
//   bit   10     in tree
//   bits 11..31  k (draws made at the node in this sample, at most kMaxDraws)
// LDS layout in 32-bit words: row offsets [n + 1], 16-bit columns [nnz]
// (padded to a whole word), then the state, node-major: word u * lanes + lane.
constexpr int64_t kLdsMaxNodes = 1024;
constexpr uint32_t kLdsTree = 1u << 10;
constexpr int kLdsKShift = 11;
static_assert(kLdsMaxNodes <= (int64_t)kLdsTree, "next must fit below the tree bit");
static_assert(((uint64_t)kMaxDraws << kLdsKShift) <= 0xFFFFFFFFull, "k must fit above the tree bit");

__host__ __device__ inline int64_t lds_state_offset(int64_t n, int64_t nnz) { return (n + 1) + (nnz + 1) / 2; }
__host__ __device__ inline int64_t lds_bytes(int64_t n, int64_t nnz, int64_t lanes) {
    return 4 * (lds_state_offset(n, nnz) + n * lanes);
}

// ------------------------------------------------------------ error reporting
enum : int32_t { kErrNone = 0, kErrDrawOverflow = 1, kErrTimeout = 2, kErrInconsistent = 3 };

struct DevErr {
    int32_t code;
    int32_t detail;
};

__device__ __forceinline__ void raise_err(DevErr *e, int32_t code, int32_t detail) {
    if (atomicCAS(&e->code, 0, code) == 0) e->detail = detail;
}
__device__ __forceinline__ bool err_set(const DevErr *e) {
    return __hip_atomic_load(&e->code, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

// ------------------------------------------------------------ kernel parameters
constexpr int kMaxKeep = 64;
constexpr int kStatIters = 0, kStatDraws = 1, kStatTrees = 2, kStatPops = 3, kStatRescans = 4,
              kStatAbsorbed = 5, kStatIdleLanes = 6, kStatParkedLanes = 7, kNumStats = 8;

struct WilsonParams {
    int64_t n, nnz;
    int64_t n_slots;       // sample slots allocated in state / slot_epoch
    const uint64_t *nbr;   // [n] packed offset/degree
    const int32_t *col;    // [2m]
    const ulonglong2 *arcs;   // [2m] {target, target's adjacency record}, or null
    int32_t root;
    uint64_t k0, k1, qid;  // Philox key and counter word 3
    int64_t sample_begin, n_samples, n_total;
    int32_t n_blocks;
    uint64_t *state;       // [slots][n]
    uint32_t *slot_epoch;  // [slots]
    unsigned long long *y1;        // [B][n] or null
    int64_t *y1_per_sample;        // [n_samples] or null
    int32_t n_keep;
    int64_t keep_idx[kMaxKeep];
    int32_t *next_out;             // [n_keep][n] or null
    int32_t *draws_out;            // [n_keep][n] or null
    unsigned long long *stats;     // [kNumStats]
    DevErr *err;
    uint64_t deadline;             // wall_clock64() ticks a kernel may run before it stops
    int64_t scan_offset;           // wave form: first node the scan visits, in [0, n)
};

// One wave-cooperative Wilson sample (the device function shared by the plain
// and the batched kernels).
struct WaveSampleArgs {
    int64_t n, nnz;
    const uint64_t *nbr;
    const int32_t *col;
    const ulonglong2 *arcs = nullptr;   // read instead of col by the arc form of the samplers
    int32_t root;
    uint64_t k0, k1, qid;
    int64_t sample;
    uint64_t *st;                  // this slot's [n] state words
    uint32_t ep;                   // this sample's epoch bit
    unsigned long long *y1b;       // [n] counts of this sample's block, or null
    int32_t *keep_next, *keep_draws;   // [n] exports of this sample, or null
    DevErr *err;
    uint64_t t0, deadline;
    int64_t scan_offset;           // start position of the scan, in [0, n)
};

struct WaveStats {
    unsigned long long iters = 0, draws = 0, trees = 0, pops = 0, rescans = 0, idle = 0, parked = 0;
};

struct AbsorbedParams {
    int64_t n;
    const uint64_t *nbr;
    const int32_t *col;
    const ulonglong2 *arcs;        // [2m] {target, target's adjacency record}, or null
    int64_t nnz;
    int32_t root;
    uint64_t k0, k1, qid;
    uint32_t kinds;                // bit 0: uniform-start walks (tag 1), bit 1: stationary-start walks (tag 2)
    int64_t walk_begin, n_walks, n_total;
    int32_t n_blocks;
    unsigned long long *y2;        // [B][n] visits of the uniform-start walks, or null
    int64_t *len_u, *len_p;        // [n_walks] lengths of each kind, or null
    unsigned long long *stats;
    DevErr *err;
    uint64_t deadline;
};

}  // namespace lap
