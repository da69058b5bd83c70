// lap_sample_forests_noalloc: the integer core of lap_sample_forests for
// callers that cannot allocate device memory (code under graph capture,
// serving loops with a fixed footprint, harnesses that forbid hipMalloc).
//
// Its scratch -- the error word, the statistics, the block counts, the slot
// epochs and the Wilson walk state -- lives in one file-scope device array of
// fixed size instead of the graph handle's growable buffers.  Each device the
// library runs on holds its own copy until the process ends; host code reaches
// it only through the address hipGetSymbolAddress returns for the current
// device (the array's name is a host-side stand-in, not a device address).
// The kernels are those of lap_sample_forests, so the counts are identical.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>

#include "lap_host.h"
#include "lap_launch.h"

namespace lap {

// 64 MiB of 8-byte words.  Layout (word offsets):
//   0            DevErr
//   8 .. 15      statistics (kNumStats words)
//   32 .. 4127   samples per block (at most kNoAllocMaxBlocks)
//   4128 ..      slot epochs (32-bit, two per word), then the walk state,
//                slots x n words, starting on a 256-byte boundary
constexpr int64_t kScratchWords = (int64_t)1 << 23;
constexpr int64_t kOffErr = 0, kOffStats = 8, kOffBlocks = 32;
constexpr int32_t kNoAllocMaxBlocks = 4096;
constexpr int64_t kOffEpochs = kOffBlocks + kNoAllocMaxBlocks;
static_assert(kNumStats <= kOffBlocks - kOffStats, "statistics overlap the block counts");

static __device__ __align__(256) uint64_t scratch[kScratchWords];

namespace {

constexpr int kMaxDevices = 64;
std::mutex g_mu;
void *g_scratch[kMaxDevices] = {nullptr};

// the device address of this device's scratch, looked up once per device
int scratch_on_device(int dev, uint64_t **out) {
    if (dev < 0 || dev >= kMaxDevices) return fail(LAP_EDEVICE, "device index beyond the scratch table");
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(LAP_EDEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch[dev] = p;
    }
    *out = static_cast<uint64_t *>(g_scratch[dev]);
    return LAP_OK;
}

// cnt[b] = samples of this call in block b: i in [begin, begin + omega) with
// floor(i * B / total) == b
__global__ void block_counts_kernel(int64_t *cnt, int32_t B, int64_t begin, int64_t omega, int64_t total) {
    for (int32_t b = (int32_t)(blockIdx.x * blockDim.x + threadIdx.x); b < B; b += (int32_t)(gridDim.x * blockDim.x)) {
        const int64_t lo = ((int64_t)b * total + B - 1) / B;
        const int64_t hi = ((int64_t)(b + 1) * total + B - 1) / B;
        const int64_t c = min(hi, begin + omega) - max(lo, begin);
        cnt[b] = c > 0 ? c : 0;
    }
}

}  // namespace
}  // namespace lap

using namespace lap;

extern "C" int lap_sample_forests_noalloc(lap_graph *g, const lap_sample_args *a, lap_counts *out,
                                          void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    Resolved r;
    int rc = resolve_args(g, a, out->n_keep, out->keep_idx, r);
    if (rc != LAP_OK) return rc;
    if (!(a->want & LAP_OUT_DEVICE))
        return fail(LAP_EINVAL, "lap_sample_forests_noalloc writes device arrays only: set LAP_OUT_DEVICE");
    if (r.B > kNoAllocMaxBlocks)
        return fail(LAP_ERANGE, "n_blocks is above " + std::to_string(kNoAllocMaxBlocks) +
                                    ", the most the fixed scratch holds block counts for");
    int dev = 0;
    HIP_TRY(hipGetDevice(&dev));
    if (dev != g->device) return fail(LAP_EINVAL, "call on the device the graph was built on");
    const int64_t n = g->csr.n;
    const bool want_y1 = (a->want & LAP_WANT_Y1) && out->y1;
    const bool want_ps = (a->want & LAP_WANT_PER_SAMPLE) && out->y1_per_sample;
    r.wilson = want_y1 || want_ps || out->n_keep > 0;
    r.y2u = (a->want & LAP_WANT_Y2_UNIFORM) && (out->y2 || out->y2len_uniform);
    r.y2p = (a->want & LAP_WANT_Y2_PI) && out->y2len_pi;

    // concurrent sample slots: as many as the walk state leaves room for in
    // the scratch (each slot: n state words and half an epoch word); the LDS
    // lane form keeps its state in LDS and needs none
    const bool in_lds = r.mode == LAP_MODE_LDS;
    const int64_t room = kScratchWords - kOffEpochs - 1 - 32;   // the epoch word rounding and the alignment
    const int64_t fit = 2 * room / (2 * std::max<int64_t>(n, 1) + 1);
    if (r.wilson && !in_lds && fit < 1)
        return fail(LAP_ERANGE, "a graph of " + std::to_string(n) + " nodes needs more walk state than the " +
                                    std::to_string(kScratchWords * 8 >> 20) + " MiB fixed scratch holds (at most " +
                                    std::to_string(room - 1) + " nodes)");
    const int64_t slots = in_lds ? r.slots : std::max<int64_t>(1, std::min(r.slots, fit));

    uint64_t *sc = nullptr;
    if ((rc = scratch_on_device(dev, &sc)) != LAP_OK) return rc;
    DevErr *err = reinterpret_cast<DevErr *>(sc + kOffErr);
    unsigned long long *stats = reinterpret_cast<unsigned long long *>(sc + kOffStats);
    int64_t *blk = reinterpret_cast<int64_t *>(sc + kOffBlocks);
    const int64_t epoch_words = slots / 2 + 1;
    uint32_t *epochs = reinterpret_cast<uint32_t *>(sc + kOffEpochs);
    const int64_t off_state = (kOffEpochs + epoch_words + 31) / 32 * 32;
    uint64_t *state = sc + off_state;
    if (r.wilson && !in_lds && off_state + slots * n > kScratchWords)
        return fail(LAP_EINVAL, "scratch layout overflow");

    hipStream_t s = (hipStream_t)hip_stream;
    // the scratch keeps the last call's contents: clear what must start at zero
    HIP_TRY(launch_fill_u64(sc + kOffErr, 0ull, 1, s));
    HIP_TRY(launch_fill_u64(sc + kOffStats, 0ull, kNumStats, s));
    if (want_y1) HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t *>(out->y1), 0ull, (int64_t)r.B * n, s));
    if (r.y2u && out->y2) HIP_TRY(launch_fill_u64(reinterpret_cast<uint64_t *>(out->y2), 0ull, (int64_t)r.B * n, s));

    const double tmo = a->timeout_s > 0 ? a->timeout_s : 120.0;
    const uint64_t deadline = (uint64_t)(tmo * g->clock_khz * 1000.0);
    const uint64_t k1 = ((uint64_t)a->stream << 32) | (uint64_t)(uint32_t)r.root;

    // absorbed walks on the caller's stream (no auxiliary stream is created)
    if (r.y2u || r.y2p) {
        AbsorbedParams ap;
        std::memset(&ap, 0, sizeof ap);
        ap.n = n;
        ap.nbr = g->nbr.as<uint64_t>();
        ap.col = g->col.as<int32_t>();
        ap.arcs = (const ulonglong2 *)g->arcs.ptr;
        ap.nnz = g->csr.rp[n];
        ap.root = r.root;
        ap.k0 = a->seed;
        ap.k1 = k1;
        ap.qid = a->qid;
        ap.kinds = (r.y2u ? 1u : 0u) | (r.y2p ? 2u : 0u);
        ap.walk_begin = r.begin;
        ap.n_walks = r.omega;
        ap.n_total = r.total;
        ap.n_blocks = r.B;
        ap.y2 = r.y2u ? reinterpret_cast<unsigned long long *>(out->y2) : nullptr;
        ap.len_u = r.y2u ? out->y2len_uniform : nullptr;
        ap.len_p = r.y2p ? out->y2len_pi : nullptr;
        ap.stats = stats;
        ap.err = err;
        ap.deadline = deadline;
        HIP_TRY(launch_absorbed(ap, s));
    }
    if (r.wilson) {
        if (!in_lds) {
            HIP_TRY(launch_fill_u64(sc + kOffEpochs, 0ull, epoch_words, s));
            HIP_TRY(launch_fill_u64(state, 0ull, slots * n, s));
        }
        WilsonParams wp;
        std::memset(&wp, 0, sizeof wp);
        wp.n = n;
        wp.nnz = g->csr.rp[n];
        wp.n_slots = slots;
        wp.nbr = g->nbr.as<uint64_t>();
        wp.col = g->col.as<int32_t>();
        wp.arcs = (const ulonglong2 *)g->arcs.ptr;   // null when the graph has no arc records
        wp.root = r.root;
        wp.k0 = a->seed;
        wp.k1 = k1;
        wp.qid = a->qid;
        wp.sample_begin = r.begin;
        wp.n_samples = r.omega;
        wp.n_total = r.total;
        wp.n_blocks = r.B;
        wp.state = state;
        wp.slot_epoch = epochs;
        wp.y1 = want_y1 ? reinterpret_cast<unsigned long long *>(out->y1) : nullptr;
        wp.y1_per_sample = want_ps ? out->y1_per_sample : nullptr;
        wp.n_keep = (int32_t)out->n_keep;
        for (int64_t q = 0; q < out->n_keep; ++q) wp.keep_idx[q] = out->keep_idx[q];
        wp.next_out = out->n_keep ? out->next : nullptr;
        wp.draws_out = out->n_keep ? out->draws : nullptr;
        wp.stats = stats;
        wp.err = err;
        wp.deadline = deadline;
        wp.scan_offset = n > 0 ? ((a->schedule % n) + n) % n : 0;
        if (r.mode == LAP_MODE_LANE) {
            HIP_TRY(launch_wilson_lane(wp, slots, s));
        } else if (in_lds) {
            HIP_TRY(launch_wilson_lds(wp, r.lds_lanes, slots, s));
        } else if (r.mode == LAP_MODE_GROUP) {
            HIP_TRY(launch_wilson_group(wp, slots, r.group, s));
        } else {
            HIP_TRY(launch_wilson_wave(wp, slots, s));
        }
        if (want_y1) {
            // the kernels count draws beyond the first; add the one-per-sample baseline
            hipLaunchKernelGGL(block_counts_kernel, dim3((unsigned)((r.B + 255) / 256)), dim3(256), 0, s, blk, r.B,
                               r.begin, r.omega, r.total);
            HIP_TRY(hipGetLastError());
            HIP_TRY(launch_add_baseline(reinterpret_cast<unsigned long long *>(out->y1), n, r.root, blk, r.B, s));
        }
    }
    HIP_TRY(hipStreamSynchronize(s));
    DevErr e{0, 0};
    uint64_t st[kNumStats];
    HIP_TRY(hipMemcpy(&e, err, sizeof e, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st, stats, sizeof st, hipMemcpyDeviceToHost));
    for (int i = 0; i < kNumStats; ++i) g->last_stats[i] = (int64_t)st[i];
    return status_from_err(e);
}
