// C ABI of the library (include/lap.h): argument checking, device workspace
// management, kernel orchestration on the caller's stream, error reporting
// and optional per-kernel event timing.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lap_host.h"
#include "lap_launch.h"

using namespace lap;

extern "C" int lap_build_csr(int64_t n, int64_t n_edges, const int32_t *src, const int32_t *dst,
                             uint32_t flags, void *hip_stream, lap_graph **out) {
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    if (flags & ~(uint32_t)(LAP_KEEP_LCC | LAP_DEGREE_ORDER)) return fail(LAP_EINVAL, "unknown flag bits");
    lap_graph *g = new (std::nothrow) lap_graph();
    if (!g) return fail(LAP_ENOMEM, "host allocation failed");
    std::string err;
    int rc = build_host_csr(n, n_edges, src, dst, (flags & LAP_KEEP_LCC) != 0, g->csr, err,
                            (flags & LAP_DEGREE_ORDER) != 0);
    if (rc != LAP_OK) {
        delete g;
        return fail(rc, err);
    }
    const int64_t nn = g->csr.n, nnz = g->csr.rp[nn];
    if (nnz >= (int64_t)1 << 40) {
        delete g;
        return fail(LAP_ERANGE, "2m must be below 2^40");
    }
    std::vector<uint64_t> nbr((size_t)nn);
    for (int64_t u = 0; u < nn; ++u) {
        const int64_t d = g->csr.rp[u + 1] - g->csr.rp[u];
        if (d >= (int64_t)1 << 24) {
            delete g;
            return fail(LAP_ERANGE, "node degree must be below 2^24");
        }
        if (d > g->max_deg) {
            g->max_deg = (int32_t)d;
            g->max_deg_node = (int32_t)u;
        }
        nbr[u] = (uint64_t)g->csr.rp[u] | ((uint64_t)d << 40);
    }
    hipStream_t s = (hipStream_t)hip_stream;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        delete g;
        return fail(LAP_EDEVICE, "no HIP device");
    }
    g->device = dev;
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, dev) == hipSuccess) g->n_cu = prop.multiProcessorCount;
    int khz = 0;
    if (hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev) == hipSuccess && khz > 0)
        g->clock_khz = khz;
    int lds = 0;
    if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
        g->lds_per_block = lds;
    auto upload = [&](DevBuf &b, const void *src_, size_t bytes) -> int {
        if (b.ensure(bytes) != LAP_OK) return LAP_ENOMEM;
        if (bytes && hipMemcpyAsync(b.ptr, src_, bytes, hipMemcpyHostToDevice, s) != hipSuccess)
            return LAP_EDEVICE;
        // an empty array still gets a defined (zero) placeholder word
        if (!bytes && launch_fill_u64(b.as<uint64_t>(), 0ull, 1, s) != hipSuccess) return LAP_EDEVICE;
        return LAP_OK;
    };
    // arcs: the target of every column entry with the target's adjacency
    // record, so a walk step or a Wilson draw is one dependent load
    std::vector<uint64_t> arcs;
    if (4 * nnz >= kArcsMinColBytes) {
        arcs.resize(2 * (size_t)nnz);
        for (int64_t j = 0; j < nnz; ++j) {
            const int32_t w = g->csr.col[j];
            arcs[2 * j] = (uint64_t)(uint32_t)w;
            arcs[2 * j + 1] = nbr[w];
        }
    }
    if ((rc = upload(g->rp, g->csr.rp.data(), sizeof(int64_t) * (nn + 1))) != LAP_OK ||
        (rc = upload(g->nbr, nbr.data(), sizeof(uint64_t) * nn)) != LAP_OK ||
        (rc = upload(g->col, g->csr.col.data(), sizeof(int32_t) * (size_t)nnz)) != LAP_OK ||
        (!arcs.empty() && (rc = upload(g->arcs, arcs.data(), sizeof(uint64_t) * arcs.size())) != LAP_OK) ||
        hipStreamSynchronize(s) != hipSuccess) {
        delete g;
        return fail(rc == LAP_OK ? LAP_EDEVICE : rc, "graph upload failed");
    }
    *out = g;
    return LAP_OK;
}

extern "C" int lap_graph_info(const lap_graph *g, int64_t *n, int64_t *nnz, int32_t *max_deg_node,
                              int32_t *max_deg) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (n) *n = g->csr.n;
    if (nnz) *nnz = g->csr.rp[g->csr.n];
    if (max_deg_node) *max_deg_node = g->max_deg_node;
    if (max_deg) *max_deg = g->max_deg;
    return LAP_OK;
}

extern "C" int lap_graph_copy_csr(const lap_graph *g, int64_t *rp, int32_t *col, int32_t *old_ids) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (rp) std::memcpy(rp, g->csr.rp.data(), sizeof(int64_t) * g->csr.rp.size());
    if (col) std::memcpy(col, g->csr.col.data(), sizeof(int32_t) * g->csr.col.size());
    if (old_ids) std::memcpy(old_ids, g->csr.old_ids.data(), sizeof(int32_t) * g->csr.old_ids.size());
    return LAP_OK;
}

extern "C" void lap_graph_free(lap_graph *g) { delete g; }

extern "C" int lap_last_stats(const lap_graph *g, int64_t *wilson_steps, int64_t *absorbed_steps,
                              int64_t *trees, int64_t *iterations, int64_t *pops, int64_t *rescans,
                              int64_t *idle_lane_rounds, int64_t *parked_lane_rounds) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (wilson_steps) *wilson_steps = g->last_stats[kStatDraws];
    if (absorbed_steps) *absorbed_steps = g->last_stats[kStatAbsorbed];
    if (trees) *trees = g->last_stats[kStatTrees];
    if (iterations) *iterations = g->last_stats[kStatIters];
    if (pops) *pops = g->last_stats[kStatPops];
    if (rescans) *rescans = g->last_stats[kStatRescans];
    if (idle_lane_rounds) *idle_lane_rounds = g->last_stats[kStatIdleLanes];
    if (parked_lane_rounds) *parked_lane_rounds = g->last_stats[kStatParkedLanes];
    return LAP_OK;
}

// --------------------------------------------------------------- sampling
namespace lap {

int32_t lds_lanes(const lap_graph *g) {
    const int64_t n = g->csr.n;
    if (n > kLdsMaxNodes) return 0;
    for (int32_t lanes = 64; lanes >= 16; lanes /= 2)
        if (lds_bytes(n, g->csr.rp[n], lanes) <= g->lds_per_block) return lanes;
    return 0;
}

int resolve_args(const lap_graph *g, const lap_sample_args *a, int64_t n_keep, const int64_t *keep_idx,
                 Resolved &r, bool reads_trees) {
    const int64_t n = g->csr.n;
    if (!a) return fail(LAP_EINVAL, "args is NULL");
    if (a->n_samples < 1) return fail(LAP_EINVAL, "n_samples must be >= 1");
    if (a->root < -1 || a->root >= n) return fail(LAP_EINVAL, "root out of range");
    if (a->n_blocks < 1) return fail(LAP_EINVAL, "n_blocks must be >= 1");
    if (a->sample_begin < 0) return fail(LAP_EINVAL, "sample_begin must be >= 0");
    if (a->mode < LAP_MODE_AUTO || a->mode > LAP_MODE_LDS) return fail(LAP_EINVAL, "unknown mode");
    if (a->group != 0 && a->group != 2 && a->group != 4 && a->group != 8)
        return fail(LAP_EINVAL, "group must be 0, 2, 4 or 8");
    if (a->pool < 0) return fail(LAP_EINVAL, "pool must be >= 0");
    if (a->walks != LAP_WALKS_FRESH && a->walks != LAP_WALKS_LOOP) return fail(LAP_EINVAL, "unknown walks");
    if (a->want & ~(uint32_t)(LAP_WANT_Y1 | LAP_WANT_Y2_UNIFORM | LAP_WANT_Y2_PI | LAP_WANT_PER_SAMPLE |
                              LAP_OUT_DEVICE))
        return fail(LAP_EINVAL, "unknown want bits");
    r.omega = a->n_samples;
    r.begin = a->sample_begin;
    r.total = a->n_total ? a->n_total : a->sample_begin + a->n_samples;
    if (r.total < r.begin + r.omega) return fail(LAP_EINVAL, "n_total < sample_begin + n_samples");
    if (r.total >= (int64_t)1 << 56) return fail(LAP_EINVAL, "sample indices must stay below 2^56");
    if (a->n_blocks > r.total) return fail(LAP_EINVAL, "n_blocks exceeds the number of samples");
    if (r.total > ((int64_t)1 << 62) / a->n_blocks) return fail(LAP_EINVAL, "n_total * n_blocks too large");
    if (n_keep < 0 || n_keep > kMaxKeep) return fail(LAP_EINVAL, "n_keep must be in [0, 64]");
    for (int64_t q = 0; q < n_keep; ++q)
        if (!keep_idx || keep_idx[q] < r.begin || keep_idx[q] >= r.begin + r.omega)
            return fail(LAP_EINVAL, "keep_idx entries must be sample indices of this call");
    r.root = a->root < 0 ? g->max_deg_node : a->root;
    r.B = a->n_blocks;
    // the device holds 16 sample waves per CU; with fewer samples than that on
    // a large graph, several waves share a sample instead (workgroup form)
    const int64_t wave_slots = (int64_t)g->n_cu * 16;
    r.mode = a->mode;
    r.lds_lanes = reads_trees ? 0 : lds_lanes(g);
    if (r.mode == LAP_MODE_LDS) {
        if (reads_trees)
            return fail(LAP_EINVAL, "this call reads the Wilson trees from device memory; the LDS form keeps "
                                    "them in LDS only: use the lane, wave or workgroup form");
        if (r.lds_lanes == 0)
            return fail(LAP_ERANGE, "the LDS form takes graphs of at most " + std::to_string(kLdsMaxNodes) +
                                        " nodes whose columns and state for 16 samples fit in " +
                                        std::to_string(g->lds_per_block) + " bytes of LDS");
    }
    if (r.mode == LAP_MODE_AUTO)
        r.mode = (r.omega * 4 <= wave_slots && n >= (1 << 16)) ? LAP_MODE_GROUP : LAP_MODE_WAVE;
    r.group = 0;
    if (r.mode == LAP_MODE_GROUP) {
        r.group = a->group;
        if (r.group == 0) {
            r.group = 2;
            while (r.group < 8 && r.omega * r.group * 2 <= wave_slots) r.group *= 2;
        }
    }
    if (r.mode == LAP_MODE_LDS) {
        // concurrent samples: the pool, else all of them (state lives in LDS)
        r.slots = std::max<int64_t>(1, std::min<int64_t>(r.omega, a->pool > 0 ? a->pool : r.omega));
        return LAP_OK;
    }
    // concurrent sample slots: bounded by the samples, the pool and a state
    // budget of 48 GiB (8 bytes per node per slot)
    const int64_t per_slot = 8 * std::max<int64_t>(n, 1);
    const int64_t budget = ((int64_t)48 << 30) / per_slot;
    int64_t pool = a->pool;
    if (pool == 0)
        pool = r.mode == LAP_MODE_LANE    ? (int64_t)g->n_cu * 256
               : r.mode == LAP_MODE_GROUP ? wave_slots / r.group
                                          : wave_slots;
    r.slots = std::max<int64_t>(1, std::min({r.omega, pool, budget}));
    return LAP_OK;
}

int status_from_err(const DevErr &e) {
    switch (e.code) {
        case kErrNone:
            return LAP_OK;
        case kErrDrawOverflow:
            if (e.detail == -22) return fail(LAP_ERANGE, "a node-pair path departed 2^32-1 times from one node");
            return fail(LAP_ERANGE, "more than 2^21-1 draws at node " + std::to_string(e.detail) + " in one sample");
        case kErrTimeout:
            return fail(LAP_ERANGE, "kernel time limit exceeded");
        default:
            if (e.detail == -20 || e.detail == -21)
                return fail(LAP_EDEVICE, "a loop-included path needed a stack entry its Wilson sample did not draw");
            return fail(LAP_EDEVICE, "walker state inconsistent (tree count " + std::to_string(e.detail) + ")");
    }
}

}  // namespace lap

namespace {

int ensure_state(lap_graph *g, int64_t slots, hipStream_t s) {
    const int64_t n = g->csr.n;
    if (slots > g->state_slots || g->state_dirty) {
        const int64_t alloc = std::max(slots, g->state_slots);
        const int64_t epoch_words = alloc / 2 + 1;   // 32-bit epochs packed in 64-bit words
        if (g->state.ensure(sizeof(uint64_t) * (size_t)alloc * n) != LAP_OK ||
            g->epoch.ensure(sizeof(uint64_t) * (size_t)epoch_words) != LAP_OK)
            return fail(LAP_ENOMEM, "cannot allocate walk state");
        HIP_TRY(launch_fill_u64(g->state.as<uint64_t>(), 0ull, alloc * n, s));
        HIP_TRY(launch_fill_u64(g->epoch.as<uint64_t>(), 0ull, epoch_words, s));
        g->state_slots = alloc;
        g->state_dirty = false;
    }
    return LAP_OK;
}

struct RunOut {
    // device arrays filled by run_sampling (owned by the handle)
    unsigned long long *y1 = nullptr, *y2 = nullptr;
    int64_t *y1s = nullptr, *len_u = nullptr, *len_p = nullptr;
    int32_t *keep_next = nullptr, *keep_draws = nullptr;
};

// Wilson samples of r (and, with loop_walks false, the requested absorbed
// walks beside them on the auxiliary stream).  With loop_walks true the
// walk counts come from the loop-included paths of the same samples instead:
// every sample of a round keeps its own state slot (one wave, workgroup or
// lane per sample; as many as 48 GiB of state and path counters hold), and
// each round's trees are followed by one path per sample for each requested
// start law.
int run_sampling(lap_graph *g, const Resolved &r, const lap_sample_args *a, int64_t n_keep,
                 const int64_t *keep_idx, bool want_y1, bool want_y1s, RunOut &o, hipStream_t s, Timer &tm,
                 bool loop_walks = false) {
    const int64_t n = g->csr.n;
    const size_t bn = sizeof(uint64_t) * (size_t)r.B * n;
    if (g->err.ensure(sizeof(DevErr)) || g->stats.ensure(sizeof(uint64_t) * kNumStats))
        return fail(LAP_ENOMEM, "cannot allocate workspace");
    if (want_y1 && g->y1.ensure(bn)) return fail(LAP_ENOMEM, "cannot allocate y1");
    if (r.y2u && g->y2.ensure(bn)) return fail(LAP_ENOMEM, "cannot allocate y2");
    if (r.wilson && g->y1s.ensure(sizeof(int64_t) * r.omega)) return fail(LAP_ENOMEM, "cannot allocate y1s");
    if (r.y2u && g->len_u.ensure(sizeof(int64_t) * r.omega)) return fail(LAP_ENOMEM, "cannot allocate len");
    if (r.y2p && g->len_p.ensure(sizeof(int64_t) * r.omega)) return fail(LAP_ENOMEM, "cannot allocate len");
    if (n_keep > 0 && (g->keep_next.ensure(sizeof(int32_t) * n_keep * n) ||
                       g->keep_draws.ensure(sizeof(int32_t) * n_keep * n)))
        return fail(LAP_ENOMEM, "cannot allocate kept samples");
    HIP_TRY(launch_fill_u64(g->err.as<uint64_t>(), 0ull, 1, s));
    HIP_TRY(launch_fill_u64(g->stats.as<uint64_t>(), 0ull, kNumStats, s));
    if (want_y1) HIP_TRY(launch_fill_u64(g->y1.as<uint64_t>(), 0ull, (int64_t)r.B * n, s));
    if (r.y2u) HIP_TRY(launch_fill_u64(g->y2.as<uint64_t>(), 0ull, (int64_t)r.B * n, s));

    const double tmo = a->timeout_s > 0 ? a->timeout_s : 120.0;
    const uint64_t deadline = (uint64_t)(tmo * g->clock_khz * 1000.0);
    const uint64_t k1 = ((uint64_t)a->stream << 32) | (uint64_t)(uint32_t)r.root;

    // absorbed walks run on the auxiliary stream, overlapping the Wilson kernel
    const bool any_walks = (r.y2u || r.y2p) && !loop_walks;
    if (any_walks) {
        if (!g->aux) {
            HIP_TRY(hipStreamCreateWithFlags(&g->aux, hipStreamNonBlocking));
            HIP_TRY(hipEventCreateWithFlags(&g->ev_fork, hipEventDisableTiming));
            HIP_TRY(hipEventCreateWithFlags(&g->ev_join, hipEventDisableTiming));
        }
        HIP_TRY(hipEventRecord(g->ev_fork, s));
        HIP_TRY(hipStreamWaitEvent(g->aux, g->ev_fork, 0));
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
        ap.y2 = r.y2u ? g->y2.as<unsigned long long>() : nullptr;
        ap.len_u = r.y2u ? g->len_u.as<int64_t>() : nullptr;
        ap.len_p = r.y2p ? g->len_p.as<int64_t>() : nullptr;
        ap.stats = g->stats.as<unsigned long long>();
        ap.err = g->err.as<DevErr>();
        ap.deadline = deadline;
        tm.begin("absorbed", g->aux);
        HIP_TRY(launch_absorbed(ap, g->aux));
        tm.end(g->aux);
        HIP_TRY(hipEventRecord(g->ev_join, g->aux));
    }
    const bool loop = loop_walks && r.wilson && (r.y2u || r.y2p);
    int64_t round = r.omega;   // samples per Wilson launch
    if (loop) {
        round = std::max<int64_t>(1, std::min<int64_t>(r.omega, ((int64_t)48 << 30) / (12 * std::max<int64_t>(n, 1))));
        if (g->loop_cnt.ensure(sizeof(int32_t) * (size_t)round * n + 8))
            return fail(LAP_ENOMEM, "cannot allocate loop-included path workspace");
    }
    for (int64_t done = 0; r.wilson && done < r.omega; done += round) {
        const int64_t rows = std::min(round, r.omega - done);
        const int64_t slots = loop ? rows : std::min(r.slots, rows);
        if (r.mode != LAP_MODE_LDS) {
            int rc = ensure_state(g, slots, s);
            if (rc != LAP_OK) return rc;
        }
        WilsonParams wp;
        std::memset(&wp, 0, sizeof wp);
        wp.n = n;
        wp.nnz = g->csr.rp[n];
        wp.n_slots = slots;   // lanes, waves or workgroups taking part; <= allocated slots
        wp.nbr = g->nbr.as<uint64_t>();
        wp.col = g->col.as<int32_t>();
        wp.arcs = (const ulonglong2 *)g->arcs.ptr;   // null when the graph has no arc records
        wp.root = r.root;
        wp.k0 = a->seed;
        wp.k1 = k1;
        wp.qid = a->qid;
        wp.sample_begin = r.begin + done;
        wp.n_samples = rows;
        wp.n_total = r.total;
        wp.n_blocks = r.B;
        wp.state = g->state.as<uint64_t>();
        wp.slot_epoch = g->epoch.as<uint32_t>();
        wp.y1 = want_y1 ? g->y1.as<unsigned long long>() : nullptr;
        wp.y1_per_sample = g->y1s.as<int64_t>() + done;
        wp.n_keep = (int32_t)n_keep;
        for (int64_t q = 0; q < n_keep; ++q) wp.keep_idx[q] = keep_idx[q];
        wp.next_out = n_keep ? g->keep_next.as<int32_t>() : nullptr;
        wp.draws_out = n_keep ? g->keep_draws.as<int32_t>() : nullptr;
        wp.stats = g->stats.as<unsigned long long>();
        wp.err = g->err.as<DevErr>();
        wp.deadline = deadline;
        wp.scan_offset = n > 0 ? ((a->schedule % n) + n) % n : 0;
        if (r.mode == LAP_MODE_LANE) {
            tm.begin("wilson_lane", s);
            HIP_TRY(launch_wilson_lane(wp, wp.n_slots, s));
        } else if (r.mode == LAP_MODE_LDS) {
            tm.begin("wilson_lds", s);
            HIP_TRY(launch_wilson_lds(wp, r.lds_lanes, wp.n_slots, s));
        } else if (r.mode == LAP_MODE_GROUP) {
            tm.begin("wilson_group", s);
            HIP_TRY(launch_wilson_group(wp, wp.n_slots, r.group, s));
        } else {
            tm.begin("wilson_wave", s);
            HIP_TRY(launch_wilson_wave(wp, wp.n_slots, s));
        }
        tm.end(s);
        for (int kind = 1; loop && kind <= 2; ++kind) {
            // one loop-included path per sample of the round, through its tree
            if ((kind == 1 && !r.y2u) || (kind == 2 && !r.y2p)) continue;
            HIP_TRY(launch_fill_u64(g->loop_cnt.as<uint64_t>(), 0ull, (rows * n + 1) / 2, s));
            LoopParams lp;
            std::memset(&lp, 0, sizeof lp);
            lp.n = n;
            lp.nnz = g->csr.rp[n];
            lp.nbr = g->nbr.as<uint64_t>();
            lp.col = g->col.as<int32_t>();
            lp.root = r.root;
            lp.k0 = a->seed;
            lp.k1 = k1;
            lp.qid = a->qid;
            lp.tag = (uint32_t)kind;
            lp.state = g->state.as<uint64_t>();
            lp.slot_epoch = g->epoch.as<uint32_t>();
            lp.cnt = g->loop_cnt.as<int32_t>();
            lp.n_paths = rows;
            lp.sample_begin = r.begin + done;
            lp.n_total = r.total;
            lp.n_blocks = r.B;
            lp.y2 = kind == 1 ? g->y2.as<unsigned long long>() : nullptr;
            lp.len_out = (kind == 1 ? g->len_u.as<int64_t>() : g->len_p.as<int64_t>()) + done;
            lp.stats = g->stats.as<unsigned long long>();
            lp.err = g->err.as<DevErr>();
            lp.deadline = deadline;
            tm.begin("loop_included", s);
            HIP_TRY(launch_loop_included(lp, s));
            tm.end(s);
        }
    }
    (void)want_y1s;
    if (any_walks) HIP_TRY(hipStreamWaitEvent(s, g->ev_join, 0));
    o.y1 = want_y1 ? g->y1.as<unsigned long long>() : nullptr;
    o.y2 = r.y2u ? g->y2.as<unsigned long long>() : nullptr;
    o.y1s = r.wilson ? g->y1s.as<int64_t>() : nullptr;
    o.len_u = r.y2u ? g->len_u.as<int64_t>() : nullptr;
    o.len_p = r.y2p ? g->len_p.as<int64_t>() : nullptr;
    o.keep_next = n_keep ? g->keep_next.as<int32_t>() : nullptr;
    o.keep_draws = n_keep ? g->keep_draws.as<int32_t>() : nullptr;
    return LAP_OK;
}

// wait for the stream, then turn a device-side error into a status
int finish(lap_graph *g, hipStream_t s, Timer &tm) {
    HIP_TRY(hipStreamSynchronize(s));
    tm.collect();
    DevErr e{0, 0};
    uint64_t st[kNumStats];
    HIP_TRY(hipMemcpy(&e, g->err.ptr, sizeof e, hipMemcpyDeviceToHost));
    HIP_TRY(hipMemcpy(st, g->stats.ptr, sizeof st, hipMemcpyDeviceToHost));
    for (int i = 0; i < kNumStats; ++i) g->last_stats[i] = (int64_t)st[i];
    if (e.code != kErrNone) {
        g->state_dirty = true;
        return status_from_err(e);
    }
    return LAP_OK;
}

int copy_out(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (!dst || !bytes) return LAP_OK;
    HIP_TRY(hipMemcpyAsync(dst, src, bytes, hipMemcpyDefault, s));
    return LAP_OK;
}

}  // namespace

extern "C" int lap_sample_forests(lap_graph *g, const lap_sample_args *a, lap_counts *out, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    Resolved r;
    int rc = resolve_args(g, a, out->n_keep, out->keep_idx, r);
    if (rc != LAP_OK) return rc;
    const bool want_y1 = (a->want & LAP_WANT_Y1) && out->y1;
    r.wilson = want_y1 || ((a->want & LAP_WANT_PER_SAMPLE) && out->y1_per_sample) || out->n_keep > 0;
    r.y2u = (a->want & LAP_WANT_Y2_UNIFORM) && (out->y2 || out->y2len_uniform);
    r.y2p = (a->want & LAP_WANT_Y2_PI) && out->y2len_pi;
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    RunOut o;
    rc = run_sampling(g, r, a, out->n_keep, out->keep_idx, want_y1, true, o, s, tm);
    if (rc != LAP_OK) return rc;
    if (want_y1) {
        // the kernels count draws beyond the first; add the one-per-sample
        // baseline: block b holds the samples i of this call with
        // floor(i*B/n_total) == b
        std::vector<int64_t> cnt((size_t)r.B);
        for (int32_t b = 0; b < r.B; ++b) {
            const int64_t lo = ((int64_t)b * r.total + r.B - 1) / r.B;
            const int64_t hi = ((int64_t)(b + 1) * r.total + r.B - 1) / r.B;
            cnt[b] = std::max<int64_t>(0, std::min(hi, r.begin + r.omega) - std::max(lo, r.begin));
        }
        if (g->blkcount.ensure(sizeof(int64_t) * r.B)) return fail(LAP_ENOMEM, "cannot allocate block counts");
        HIP_TRY(hipMemcpyAsync(g->blkcount.ptr, cnt.data(), sizeof(int64_t) * r.B, hipMemcpyHostToDevice, s));
        HIP_TRY(launch_add_baseline(o.y1, g->csr.n, r.root, g->blkcount.as<int64_t>(), r.B, s));
        HIP_TRY(hipStreamSynchronize(s));   // cnt lives on this stack frame
    }
    rc = finish(g, s, tm);
    if (rc != LAP_OK) return rc;
    const int64_t n = g->csr.n;
    const size_t bn = sizeof(int64_t) * (size_t)r.B * n;
    if (want_y1 && (rc = copy_out(out->y1, o.y1, bn, s))) return rc;
    if (r.y2u && out->y2 && (rc = copy_out(out->y2, o.y2, bn, s))) return rc;
    if (r.wilson && (a->want & LAP_WANT_PER_SAMPLE) &&
        (rc = copy_out(out->y1_per_sample, o.y1s, sizeof(int64_t) * r.omega, s)))
        return rc;
    if (r.y2u && (rc = copy_out(out->y2len_uniform, o.len_u, sizeof(int64_t) * r.omega, s))) return rc;
    if (r.y2p && (rc = copy_out(out->y2len_pi, o.len_p, sizeof(int64_t) * r.omega, s))) return rc;
    if (out->n_keep > 0) {
        if ((rc = copy_out(out->next, o.keep_next, sizeof(int32_t) * out->n_keep * n, s))) return rc;
        if ((rc = copy_out(out->draws, o.keep_draws, sizeof(int32_t) * out->n_keep * n, s))) return rc;
    }
    HIP_TRY(hipStreamSynchronize(s));
    return LAP_OK;
}

extern "C" int lap_estimate(lap_graph *g, const lap_sample_args *a, lap_estimates *out, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (!out) return fail(LAP_EINVAL, "out is NULL");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, a && a->walks == LAP_WALKS_LOOP);
    if (rc != LAP_OK) return rc;
    if (r.begin != 0 || r.total != r.omega)
        return fail(LAP_EINVAL, "lap_estimate runs a whole sample set: sample_begin = 0, n_total = n_samples");
    const bool want_diag = out->diag || out->diag_se || out->lv_diag || out->closeness || out->trace ||
                           out->kirchhoff || out->rw_betweenness;
    const bool want_kem = out->kemeny || out->kemeny_se;
    if (!want_diag && !want_kem) return LAP_OK;
    r.wilson = true;
    r.y2u = want_diag;
    r.y2p = want_kem;
    hipStream_t s = (hipStream_t)hip_stream;
    const int64_t n = g->csr.n;
    Timer tm;
    RunOut o;
    rc = run_sampling(g, r, a, 0, nullptr, want_diag, true, o, s, tm, a->walks == LAP_WALKS_LOOP);
    if (rc != LAP_OK) return rc;
    // FP64 assembly on the device into handle-owned buffers
    const int32_t parts = (int32_t)std::min<int64_t>(1024, std::max<int64_t>(1, (n + 1023) / 1024));
    if (g->asm_partial.ensure(sizeof(double) * (size_t)(r.B + 1) * parts) ||
        g->asm_sums.ensure(sizeof(double) * (size_t)(r.B + 2)) || g->asm_trace.ensure(sizeof(double) * parts) ||
        g->est_out.ensure(sizeof(double) * (5 * (size_t)n + 5)))
        return fail(LAP_ENOMEM, "cannot allocate assembly buffers");
    double *d_diag = g->est_out.as<double>(), *d_se = d_diag + n, *d_lv = d_se + n, *d_c = d_lv + n;
    double *d_rwb = d_c + n;
    double *d_scal = d_rwb + n;   // trace, kappa, kappa_se, kirchhoff
    tm.begin("assemble", s);
    if (want_diag) {
        AssembleParams ap;
        std::memset(&ap, 0, sizeof ap);
        ap.n = n;
        ap.root = r.root;
        ap.n_blocks = r.B;
        ap.omega = r.omega;
        ap.nbr = g->nbr.as<uint64_t>();
        ap.y1 = o.y1;
        ap.y2 = o.y2;
        ap.partial = g->asm_partial.as<double>();
        ap.sums = g->asm_sums.as<double>();
        ap.trace_parts = g->asm_trace.as<double>();
        ap.diag = d_diag;
        ap.diag_se = d_se;
        ap.lv_diag = d_lv;
        ap.closeness = d_c;
        ap.rw_betweenness = d_rwb;
        ap.trace = d_scal;
        ap.kirchhoff = d_scal + 3;
        ap.n_parts = parts;
        HIP_TRY(launch_assemble_diag(ap, s));
    }
    if (want_kem) HIP_TRY(launch_kemeny(o.y1s, o.len_p, r.omega, d_scal + 1, d_scal + 2, s));
    tm.end(s);
    rc = finish(g, s, tm);
    if (rc != LAP_OK) return rc;
    if (n == 1) {
        // a single node: every estimate is zero
        std::vector<double> z(5 * (size_t)n + 5, 0.0);
        HIP_TRY(hipMemcpy(d_diag, z.data(), z.size() * sizeof(double), hipMemcpyHostToDevice));
    }
    if ((rc = copy_out(out->diag, d_diag, sizeof(double) * n, s)) ||
        (rc = copy_out(out->diag_se, d_se, sizeof(double) * n, s)) ||
        (rc = copy_out(out->lv_diag, d_lv, sizeof(double) * n, s)) ||
        (rc = copy_out(out->closeness, d_c, sizeof(double) * n, s)) ||
        (rc = copy_out(out->trace, d_scal, sizeof(double), s)) ||
        (rc = copy_out(out->kemeny, d_scal + 1, sizeof(double), s)) ||
        (rc = copy_out(out->kemeny_se, d_scal + 2, sizeof(double), s)) ||
        (rc = copy_out(out->kirchhoff, d_scal + 3, sizeof(double), s)) ||
        (rc = copy_out(out->rw_betweenness, d_rwb, sizeof(double) * n, s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return LAP_OK;
}

// ---------------------------------------------------------------- SpanTree
namespace {

// Wilson trees for the samples of r, `slots` at a time, each round followed by
// the SpanTree pass over the trees in the state slots.  Fills g->span_x
// (X1 then X2, [B][n] each) and g->span_s (s1 then s2, [omega] each).
int span_run(lap_graph *g, const lap_sample_args *a, const Resolved &r, hipStream_t s, Timer &tm) {
    const int64_t n = g->csr.n;
    if (g->bfs_root != r.root) {
        std::vector<int32_t> par;
        if (bfs_parents(g->csr, r.root, par) != n) return fail(LAP_ENOTCONN, "graph is not connected");
        if (g->bfs_par.ensure(sizeof(int32_t) * (size_t)n)) return fail(LAP_ENOMEM, "cannot allocate BFS tree");
        HIP_TRY(hipMemcpyAsync(g->bfs_par.ptr, par.data(), sizeof(int32_t) * (size_t)n, hipMemcpyHostToDevice, s));
        HIP_TRY(hipStreamSynchronize(s));   // par lives on this stack frame
        g->bfs_root = r.root;
    }
    // trees per round: the sampling slots, within 48 GiB of tree scratch
    const int64_t per_tree = (8 * kSpanInt64PerNode + 4 * kSpanInt32PerNode) * std::max<int64_t>(n, 1);
    const int64_t slots = std::max<int64_t>(1, std::min<int64_t>(r.slots, ((int64_t)48 << 30) / per_tree));
    if (g->span64.ensure(sizeof(int64_t) * (size_t)kSpanInt64PerNode * slots * n) ||
        g->span32.ensure(sizeof(int32_t) * (size_t)kSpanInt32PerNode * slots * n) ||
        g->span_x.ensure(sizeof(uint64_t) * 2 * (size_t)r.B * n) ||
        g->span_s.ensure(sizeof(int64_t) * 2 * (size_t)r.omega))
        return fail(LAP_ENOMEM, "cannot allocate SpanTree workspace");
    HIP_TRY(launch_fill_u64(g->span_x.as<uint64_t>(), 0ull, 2 * (int64_t)r.B * n, s));
    int64_t acc[kNumStats] = {0};
    for (int64_t done = 0; done < r.omega; done += slots) {
        Resolved rr = r;
        rr.omega = std::min(slots, r.omega - done);
        rr.begin = r.begin + done;
        rr.slots = rr.omega;
        rr.wilson = true;
        rr.y2u = rr.y2p = false;
        RunOut o;
        int rc = run_sampling(g, rr, a, 0, nullptr, false, false, o, s, tm);
        if (rc != LAP_OK) return rc;
        SpanParams p;
        std::memset(&p, 0, sizeof p);
        p.n = n;
        p.nbr = g->nbr.as<uint64_t>();
        p.root = r.root;
        p.state = g->state.as<uint64_t>();
        p.n_trees = rr.omega;
        p.sample_begin = rr.begin;
        p.n_total = r.total;
        p.n_blocks = r.B;
        p.bfs_par = g->bfs_par.as<int32_t>();
        p.scratch64 = g->span64.as<int64_t>();
        p.scratch32 = g->span32.as<int32_t>();
        p.X1 = g->span_x.as<unsigned long long>();
        p.X2 = p.X1 + (int64_t)r.B * n;
        p.s1 = g->span_s.as<long long>() + done;
        p.s2 = g->span_s.as<long long>() + r.omega + done;
        p.err = g->err.as<DevErr>();
        tm.begin("spantree", s);
        HIP_TRY(launch_spantree(p, s));
        tm.end(s);
        rc = finish(g, s, tm);
        if (rc != LAP_OK) return rc;
        for (int i = 0; i < kNumStats; ++i) acc[i] += g->last_stats[i];
    }
    for (int i = 0; i < kNumStats; ++i) g->last_stats[i] = acc[i];
    return LAP_OK;
}

}  // namespace

extern "C" int lap_spantree(lap_graph *g, const lap_sample_args *a, int64_t *X1, int64_t *X2, int64_t *s1,
                            int64_t *s2, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, true);
    if (rc != LAP_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    if ((rc = span_run(g, a, r, s, tm)) != LAP_OK) return rc;
    const int64_t n = g->csr.n;
    const size_t bn = sizeof(int64_t) * (size_t)r.B * n;
    const int64_t *x = g->span_x.as<int64_t>(), *ps = g->span_s.as<int64_t>();
    if ((rc = copy_out(X1, x, bn, s)) || (rc = copy_out(X2, x + (int64_t)r.B * n, bn, s)) ||
        (rc = copy_out(s1, ps, sizeof(int64_t) * r.omega, s)) ||
        (rc = copy_out(s2, ps + r.omega, sizeof(int64_t) * r.omega, s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return LAP_OK;
}

extern "C" int lap_spantree_estimate(lap_graph *g, const lap_sample_args *a, double *diag, double *diag_se,
                                     double *closeness, double *kemeny, double *kemeny_se, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, true);
    if (rc != LAP_OK) return rc;
    if (r.begin != 0 || r.total != r.omega)
        return fail(LAP_EINVAL, "a SpanTree estimate runs a whole sample set: sample_begin = 0, n_total = n_samples");
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    if ((rc = span_run(g, a, r, s, tm)) != LAP_OK) return rc;
    const int64_t n = g->csr.n;
    std::vector<int64_t> bn((size_t)r.B);
    for (int32_t b = 0; b < r.B; ++b)
        bn[b] = ((int64_t)(b + 1) * r.total + r.B - 1) / r.B - ((int64_t)b * r.total + r.B - 1) / r.B;
    // device outputs: diag, diag_se, closeness [n]; trace, kemeny, kemeny_se; partial traces;
    // block sizes and sums
    const int64_t parts = span_assemble_parts(n);
    if (g->est_out.ensure(sizeof(double) * (3 * (size_t)n + 3 + (size_t)parts) + 2 * sizeof(int64_t) * (size_t)r.B))
        return fail(LAP_ENOMEM, "cannot allocate estimates");
    double *d = g->est_out.as<double>();
    int64_t *blk = (int64_t *)(d + 3 * n + 3 + parts);
    HIP_TRY(hipMemcpyAsync(blk, bn.data(), sizeof(int64_t) * r.B, hipMemcpyHostToDevice, s));
    SpanAsmParams p;
    std::memset(&p, 0, sizeof p);
    p.n = n;
    p.omega = r.omega;
    p.two_m = g->csr.rp[n];
    p.B = r.B;
    p.X1 = g->span_x.as<unsigned long long>();
    p.X2 = p.X1 + (int64_t)r.B * n;
    p.blk_n = blk;
    p.blk_sum = (long long *)(blk + r.B);
    p.s1 = g->span_s.as<long long>();
    p.s2 = p.s1 + r.omega;
    const bool want_diag = diag || diag_se || closeness;
    p.diag = want_diag ? d : nullptr;
    p.diag_se = diag_se ? d + n : nullptr;
    p.closeness = closeness ? d + 2 * n : nullptr;
    p.trace = d + 3 * n;
    p.kemeny = (kemeny || kemeny_se) ? d + 3 * n + 1 : nullptr;
    p.kemeny_se = kemeny_se ? d + 3 * n + 2 : nullptr;
    p.part = d + 3 * n + 3;
    p.n_parts = parts;
    HIP_TRY(launch_span_assemble(p, s));
    if ((rc = copy_out(diag, d, sizeof(double) * n, s)) || (rc = copy_out(diag_se, d + n, sizeof(double) * n, s)) ||
        (rc = copy_out(closeness, d + 2 * n, sizeof(double) * n, s)) ||
        (rc = copy_out(kemeny, d + 3 * n + 1, sizeof(double), s)) ||
        (rc = copy_out(kemeny_se, d + 3 * n + 2, sizeof(double), s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));   // bn lives on this stack frame
    return LAP_OK;
}

// ------------------------------------------------------ loop-included paths
extern "C" int lap_loop_included(lap_graph *g, const lap_sample_args *a, int32_t tag, int64_t *Y2, int64_t *len,
                                 void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (tag != 1 && tag != 2) return fail(LAP_EINVAL, "tag must be 1 (uniform start) or 2 (stationary start)");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, true);
    if (rc != LAP_OK) return rc;
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    const int64_t n = g->csr.n;
    const int64_t slots =
        std::max<int64_t>(1, std::min<int64_t>(r.slots, ((int64_t)48 << 30) / (4 * std::max<int64_t>(n, 1))));
    if (g->loop_cnt.ensure(sizeof(int32_t) * (size_t)slots * n + 8) ||
        g->loop_y2.ensure(sizeof(uint64_t) * (size_t)r.B * n) || g->loop_len.ensure(sizeof(int64_t) * r.omega))
        return fail(LAP_ENOMEM, "cannot allocate loop-included path workspace");
    HIP_TRY(launch_fill_u64(g->loop_y2.as<uint64_t>(), 0ull, (int64_t)r.B * n, s));
    const double tmo = a->timeout_s > 0 ? a->timeout_s : 120.0;
    int64_t acc[kNumStats] = {0};
    for (int64_t done = 0; done < r.omega; done += slots) {
        Resolved rr = r;
        rr.omega = std::min(slots, r.omega - done);
        rr.begin = r.begin + done;
        rr.slots = rr.omega;
        rr.wilson = true;
        rr.y2u = rr.y2p = false;
        RunOut o;
        if ((rc = run_sampling(g, rr, a, 0, nullptr, false, false, o, s, tm)) != LAP_OK) return rc;
        HIP_TRY(launch_fill_u64(g->loop_cnt.as<uint64_t>(), 0ull, (rr.omega * n + 1) / 2, s));
        LoopParams p;
        std::memset(&p, 0, sizeof p);
        p.n = n;
        p.nnz = g->csr.rp[n];
        p.nbr = g->nbr.as<uint64_t>();
        p.col = g->col.as<int32_t>();
        p.root = r.root;
        p.k0 = a->seed;
        p.k1 = ((uint64_t)a->stream << 32) | (uint64_t)(uint32_t)r.root;
        p.qid = a->qid;
        p.tag = (uint32_t)tag;
        p.state = g->state.as<uint64_t>();
        p.slot_epoch = g->epoch.as<uint32_t>();
        p.cnt = g->loop_cnt.as<int32_t>();
        p.n_paths = rr.omega;
        p.sample_begin = rr.begin;
        p.n_total = r.total;
        p.n_blocks = r.B;
        p.y2 = g->loop_y2.as<unsigned long long>();
        p.len_out = g->loop_len.as<int64_t>() + done;
        p.err = g->err.as<DevErr>();
        p.deadline = (uint64_t)(tmo * g->clock_khz * 1000.0);
        tm.begin("loop_included", s);
        HIP_TRY(launch_loop_included(p, s));
        tm.end(s);
        if ((rc = finish(g, s, tm)) != LAP_OK) return rc;
        for (int i = 0; i < kNumStats; ++i) acc[i] += g->last_stats[i];
    }
    for (int i = 0; i < kNumStats; ++i) g->last_stats[i] = acc[i];
    if ((rc = copy_out(Y2, g->loop_y2.ptr, sizeof(int64_t) * (size_t)r.B * n, s)) ||
        (rc = copy_out(len, g->loop_len.ptr, sizeof(int64_t) * r.omega, s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    return LAP_OK;
}

// ------------------------------------------- loop-included paths, node pairs
namespace {

constexpr int32_t kPairHashLog2 = 14;              // 16384-word table per lane (128 KiB)
constexpr int64_t kPairMaxLanes = (int64_t)1 << 17;
constexpr int64_t kPairMaxPairs = (int64_t)1 << 23;
constexpr int64_t kPairCountBudget = (int64_t)32 << 30;   // bytes of departure counters per form

// Count words and last tags for `lanes` lanes of `words` words each; lanes
// beyond those already set up (all of them after a reallocation) start zeroed.
int ready_lanes(DevBuf &words_buf, DevBuf &tags_buf, int64_t &ready, int64_t lanes, int64_t words,
                hipStream_t s) {
    if (lanes <= ready) return LAP_OK;
    if (words_buf.ensure(sizeof(uint64_t) * (size_t)lanes * words + 8) ||
        tags_buf.ensure(sizeof(uint32_t) * (size_t)lanes + 8))
        return fail(LAP_ENOMEM, "cannot allocate pair path counters");
    HIP_TRY(launch_fill_u64(words_buf.as<uint64_t>(), 0ull, lanes * words, s));
    HIP_TRY(launch_fill_u64(tags_buf.as<uint64_t>(), 0ull, (lanes + 1) / 2, s));
    ready = lanes;
    return LAP_OK;
}

}  // namespace

namespace {

// The launches of lap_pair_paths (rows null: paths from s_j and from t_j,
// sums into pair_v) and of lap_lv_rows (rows given: one path from each s_j,
// departures per node into rows).  d_ids holds s (and t) on the device.
int pair_run(lap_graph *g, const Resolved &r, const lap_sample_args *a, const int32_t *d_ids, int64_t n_pairs,
             unsigned long long *rows, int32_t check, int64_t lanes, hipStream_t s, Timer &tm) {
    int rc = LAP_OK;
    const int64_t n = g->csr.n;
    const int64_t paths = rows ? n_pairs : 2 * n_pairs;
    const int64_t hash_words = (int64_t)1 << kPairHashLog2;
    // Lanes in flight: bounded by the counter budget and by `lanes`.  Graphs
    // with more nodes than a table has words use the hashed form first.
    auto lane_cap = [&](int64_t words) {
        int64_t c = std::min<int64_t>(kPairCountBudget / (8 * words), kPairMaxLanes);
        if (lanes > 0) c = std::min(c, lanes);
        return std::max<int64_t>(c, 1);
    };
    const int64_t dense_cap = lane_cap(std::max<int64_t>(n, 1));
    const int64_t hash_cap = lane_cap(hash_words);
    bool hashed = n > hash_words;
    if (g->pair_next.ensure(sizeof(uint64_t) * 128) || g->pair_v.ensure(sizeof(uint64_t) * 4) ||
        g->err.ensure(sizeof(DevErr)) || g->stats.ensure(sizeof(uint64_t) * kNumStats))
        return fail(LAP_ENOMEM, "cannot allocate pair path workspace");
    const double tmo = a->timeout_s > 0 ? a->timeout_s : 120.0;
    int64_t acc[kNumStats] = {0};
    int64_t queued_total = 0, hashed_items = 0;
    auto run = [&](PairParams &p, bool hash_form, int64_t L) -> int {
        p.n_lanes = L;
        p.n_parts = (int32_t)std::min<int64_t>(8, (L + 63) / 64);
        HIP_TRY(launch_fill_u64(g->pair_next.as<uint64_t>(), 0ull, 128, s));
        tm.begin("pair_paths", s);
        HIP_TRY(launch_pair_paths(p, hash_form, s));
        tm.end(s);
        int rc2 = finish(g, s, tm);
        if (rc2 != LAP_OK) return rc2;
        for (int k = 0; k < kNumStats; ++k) acc[k] += g->last_stats[k];
        return LAP_OK;
    };
    for (int64_t done = 0; done < r.omega;) {
        // samples of this launch: all of them, within the Wilson slots when
        // checking, and within the queue's capacity in the hashed form
        int64_t chunk = r.omega - done;
        if (check) chunk = std::min(chunk, r.slots);
        if (hashed) chunk = std::max<int64_t>(1, std::min(chunk, (2 * kPairMaxPairs) / paths));
        const int64_t items = chunk * paths;
        PairParams p;
        std::memset(&p, 0, sizeof p);
        if (check) {
            Resolved rr = r;
            rr.omega = chunk;
            rr.begin = r.begin + done;
            rr.slots = chunk;
            rr.wilson = true;
            rr.y2u = rr.y2p = false;
            RunOut o;
            if ((rc = run_sampling(g, rr, a, 0, nullptr, false, false, o, s, tm)) != LAP_OK) return rc;
            p.state = g->state.as<uint64_t>();
            p.slot_epoch = g->epoch.as<uint32_t>();
        } else {
            HIP_TRY(launch_fill_u64(g->err.as<uint64_t>(), 0ull, 1, s));
            HIP_TRY(launch_fill_u64(g->stats.as<uint64_t>(), 0ull, kNumStats, s));
        }
        p.n = n;
        p.nbr = g->nbr.as<uint64_t>();
        p.col = g->col.as<int32_t>();
        p.root = r.root;
        p.k0 = a->seed;
        p.k1 = ((uint64_t)a->stream << 32) | (uint64_t)(uint32_t)r.root;
        p.qid = a->qid;
        p.ps = d_ids;
        p.pt = d_ids + n_pairs;
        p.n_pairs = n_pairs;
        p.n_items = items;
        p.next = g->pair_next.as<unsigned long long>();
        p.sample_begin = r.begin + done;
        p.n_total = r.total;
        p.n_blocks = r.B;
        p.V = g->pair_v.as<unsigned long long>();
        p.rows = rows;
        p.stats = g->stats.as<unsigned long long>();
        p.err = g->err.as<DevErr>();
        p.deadline = (uint64_t)(tmo * g->clock_khz * 1000.0);
        if (hashed) {
            const int64_t L = std::min(hash_cap, items);
            if ((rc = ready_lanes(g->pair_tbl, g->pair_tbl_tags, g->pair_tbl_lanes, L, hash_words, s)) != LAP_OK)
                return rc;
            if (g->pair_queue.ensure(sizeof(uint64_t) * (size_t)(items + 1)))
                return fail(LAP_ENOMEM, "cannot allocate pair path queue");
            p.tbl = g->pair_tbl.as<uint64_t>();
            p.lane_tag = g->pair_tbl_tags.as<uint32_t>();
            p.hash_log2 = kPairHashLog2;
            p.hash_limit = (int32_t)(hash_words * 3 / 4);
            p.queue_out_len = g->pair_queue.as<unsigned long long>();
            p.queue_out = p.queue_out_len + 1;
            HIP_TRY(launch_fill_u64((uint64_t *)p.queue_out_len, 0ull, 1, s));
            if ((rc = run(p, true, L)) != LAP_OK) return rc;
            // paths that filled their table run again in the dense form
            unsigned long long queued = 0;
            HIP_TRY(hipMemcpy(&queued, p.queue_out_len, sizeof queued, hipMemcpyDeviceToHost));
            hashed_items += items;
            queued_total += (int64_t)queued;
            if (queued > 0) {
                const int64_t Ld = std::min<int64_t>(dense_cap, (int64_t)queued);
                if ((rc = ready_lanes(g->pair_cnt, g->pair_cnt_tags, g->pair_cnt_lanes, Ld, n, s)) != LAP_OK)
                    return rc;
                HIP_TRY(launch_fill_u64(g->err.as<uint64_t>(), 0ull, 1, s));
                HIP_TRY(launch_fill_u64(g->stats.as<uint64_t>(), 0ull, kNumStats, s));
                PairParams d = p;
                d.tbl = nullptr;
                d.cnt = g->pair_cnt.as<uint64_t>();
                d.lane_tag = g->pair_cnt_tags.as<uint32_t>();
                d.queue_in = p.queue_out;
                d.queue_in_len = p.queue_out_len;
                d.queue_out = d.queue_out_len = nullptr;
                if ((rc = run(d, false, Ld)) != LAP_OK) return rc;
            }
            // when many paths outgrow the tables, the dense form takes the rest
            if (queued_total * 4 > hashed_items) hashed = false;
        } else {
            const int64_t L = std::min(dense_cap, items);
            if ((rc = ready_lanes(g->pair_cnt, g->pair_cnt_tags, g->pair_cnt_lanes, L, n, s)) != LAP_OK) return rc;
            p.cnt = g->pair_cnt.as<uint64_t>();
            p.lane_tag = g->pair_cnt_tags.as<uint32_t>();
            if ((rc = run(p, false, L)) != LAP_OK) return rc;
        }
        done += chunk;
    }
    for (int i = 0; i < kNumStats; ++i) g->last_stats[i] = acc[i];
    return LAP_OK;
}

}  // namespace

extern "C" int lap_pair_paths(lap_graph *g, const lap_sample_args *a, const int32_t *ps, const int32_t *pt,
                              int64_t n_pairs, int32_t check, int64_t lanes, int64_t *V, double *r_out,
                              double *r_se, double *lv, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (n_pairs < 1 || n_pairs > kPairMaxPairs) return fail(LAP_EINVAL, "n_pairs must be in [1, 2^23]");
    if (!ps || !pt) return fail(LAP_EINVAL, "pair arrays are NULL");
    if (check != 0 && check != 1) return fail(LAP_EINVAL, "check must be 0 or 1");
    if (lanes < 0) return fail(LAP_EINVAL, "lanes must be >= 0");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, true);
    if (rc != LAP_OK) return rc;
    const int64_t n = g->csr.n;
    for (int64_t j = 0; j < n_pairs; ++j)
        if (ps[j] < 0 || ps[j] >= n || pt[j] < 0 || pt[j] >= n) return fail(LAP_EINVAL, "pair node out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    const size_t vwords = (size_t)r.B * n_pairs * 4;
    if (g->pair_ids.ensure(sizeof(int32_t) * (size_t)(2 * n_pairs)) || g->pair_v.ensure(sizeof(uint64_t) * vwords) ||
        g->pair_out.ensure(sizeof(double) * (size_t)n_pairs * 5))
        return fail(LAP_ENOMEM, "cannot allocate pair path workspace");
    int32_t *d_ids = g->pair_ids.as<int32_t>();
    HIP_TRY(hipMemcpyAsync(d_ids, ps, sizeof(int32_t) * n_pairs, hipMemcpyHostToDevice, s));
    HIP_TRY(hipMemcpyAsync(d_ids + n_pairs, pt, sizeof(int32_t) * n_pairs, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u64(g->pair_v.as<uint64_t>(), 0ull, (int64_t)vwords, s));
    if ((rc = pair_run(g, r, a, d_ids, n_pairs, nullptr, check, lanes, s, tm)) != LAP_OK) return rc;
    double *d = g->pair_out.as<double>();
    PairAsmParams q;
    q.nbr = g->nbr.as<uint64_t>();
    q.ps = d_ids;
    q.pt = d_ids + n_pairs;
    q.n_pairs = n_pairs;
    q.omega = r.omega;
    q.B = r.B;
    q.V = g->pair_v.as<unsigned long long>();
    q.r = d;
    q.r_se = d + n_pairs;
    q.lv = d + 2 * n_pairs;
    tm.begin("pair_assemble", s);
    HIP_TRY(launch_pair_assemble(q, s));
    tm.end(s);
    if ((rc = copy_out(V, g->pair_v.ptr, sizeof(int64_t) * vwords, s)) ||
        (rc = copy_out(r_out, d, sizeof(double) * n_pairs, s)) ||
        (rc = copy_out(r_se, d + n_pairs, sizeof(double) * n_pairs, s)) ||
        (rc = copy_out(lv, d + 2 * n_pairs, sizeof(double) * 3 * n_pairs, s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    tm.collect();
    return LAP_OK;
}


extern "C" int lap_lv_rows(lap_graph *g, const lap_sample_args *a, const int32_t *sources, int64_t n_sources,
                           int32_t check, int64_t lanes, int64_t *Y, double *rows, void *hip_stream) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    if (n_sources < 1 || n_sources > kPairMaxPairs) return fail(LAP_EINVAL, "n_sources must be in [1, 2^23]");
    if (!sources) return fail(LAP_EINVAL, "source array is NULL");
    if (check != 0 && check != 1) return fail(LAP_EINVAL, "check must be 0 or 1");
    if (lanes < 0) return fail(LAP_EINVAL, "lanes must be >= 0");
    Resolved r;
    int rc = resolve_args(g, a, 0, nullptr, r, true);
    if (rc != LAP_OK) return rc;
    const int64_t n = g->csr.n;
    for (int64_t j = 0; j < n_sources; ++j)
        if (sources[j] < 0 || sources[j] >= n) return fail(LAP_EINVAL, "source node out of range");
    hipStream_t s = (hipStream_t)hip_stream;
    Timer tm;
    const int64_t ywords = (int64_t)r.B * n_sources * n;
    if (ywords > ((int64_t)8 << 30)) return fail(LAP_ENOMEM, "B * n_sources * n exceeds 2^33 counts");
    if (g->pair_ids.ensure(sizeof(int32_t) * (size_t)n_sources) || g->pair_rows.ensure(sizeof(uint64_t) * ywords) ||
        g->pair_rows_out.ensure(sizeof(double) * (size_t)(n_sources * n)))
        return fail(LAP_ENOMEM, "cannot allocate row workspace");
    int32_t *d_ids = g->pair_ids.as<int32_t>();
    HIP_TRY(hipMemcpyAsync(d_ids, sources, sizeof(int32_t) * n_sources, hipMemcpyHostToDevice, s));
    HIP_TRY(launch_fill_u64(g->pair_rows.as<uint64_t>(), 0ull, ywords, s));
    unsigned long long *Yd = g->pair_rows.as<unsigned long long>();
    if ((rc = pair_run(g, r, a, d_ids, n_sources, Yd, check, lanes, s, tm)) != LAP_OK) return rc;
    double *out = g->pair_rows_out.as<double>();
    tm.begin("lv_rows", s);
    HIP_TRY(launch_lv_rows(Yd, g->nbr.as<uint64_t>(), n, n_sources, r.B, r.omega, r.root, out, s));
    tm.end(s);
    if ((rc = copy_out(Y, Yd, sizeof(int64_t) * (size_t)ywords, s)) ||
        (rc = copy_out(rows, out, sizeof(double) * (size_t)(n_sources * n), s)))
        return rc;
    HIP_TRY(hipStreamSynchronize(s));
    tm.collect();
    return LAP_OK;
}

// ------------------------------------------------ SpanTree sample bounds
extern "C" int lap_spantree_sample_bound(const lap_graph *g, int32_t root, int32_t kind, double eps, double p_fail,
                                         double *omega, int32_t *depth) {
    if (!g) return fail(LAP_EINVAL, "graph is NULL");
    const int64_t n = g->csr.n;
    if (root < -1 || root >= n) return fail(LAP_EINVAL, "root out of range");
    if (kind != 1 && kind != 2) return fail(LAP_EINVAL, "kind must be 1 (closeness) or 2 (Kemeny)");
    if (!(eps > 0.0) || !(p_fail > 0.0) || !(p_fail < 1.0)) return fail(LAP_EINVAL, "need eps > 0 and 0 < p_fail < 1");
    const int32_t v = root < 0 ? g->max_deg_node : root;
    // depth of the BFS tree from v: the longest BFS path any flow is sent along
    std::vector<int32_t> dist((size_t)n, -1), queue;
    queue.reserve((size_t)n);
    dist[v] = 0;
    queue.push_back(v);
    int32_t D = 0;
    for (size_t h = 0; h < queue.size(); ++h) {
        const int32_t a = queue[h];
        D = std::max(D, dist[a]);
        for (int64_t j = g->csr.rp[a]; j < g->csr.rp[a + 1]; ++j) {
            const int32_t b = g->csr.col[j];
            if (dist[b] < 0) {
                dist[b] = dist[a] + 1;
                queue.push_back(b);
            }
        }
    }
    const double m = 0.5 * (double)g->csr.rp[n];
    const double d2 = (double)D * (double)D;
    const double w = (kind == 1) ? 32.0 * d2 * std::log(2.0 * (double)n / p_fail) / (eps * eps)
                                 : 8.0 * m * m * d2 * std::log(2.0 / p_fail) / (eps * eps);
    if (omega) *omega = std::ceil(w);
    if (depth) *depth = D;
    return LAP_OK;
}

static lap_sample_args default_args(int32_t root, int64_t omega, uint64_t seed, int32_t B) {
    lap_sample_args a;
    std::memset(&a, 0, sizeof a);
    a.n_samples = omega;
    a.seed = seed;
    a.root = root;
    a.n_blocks = B;
    return a;
}

extern "C" int lap_diag_Ldagger(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *diag,
                                double *se, void *hip_stream) {
    const int32_t B = se ? (int32_t)std::min<int64_t>(64, std::max<int64_t>(omega, 1)) : 1;
    lap_sample_args a = default_args(root, omega, seed, B);
    lap_estimates e;
    std::memset(&e, 0, sizeof e);
    e.diag = diag;
    e.diag_se = se;
    if (!diag && !se) return fail(LAP_EINVAL, "no output requested");
    return lap_estimate(g, &a, &e, hip_stream);
}

extern "C" int lap_ecc(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *c,
                       double *trace_Ldagger, void *hip_stream) {
    lap_sample_args a = default_args(root, omega, seed, 1);
    lap_estimates e;
    std::memset(&e, 0, sizeof e);
    e.closeness = c;
    e.trace = trace_Ldagger;
    if (!c && !trace_Ldagger) return fail(LAP_EINVAL, "no output requested");
    return lap_estimate(g, &a, &e, hip_stream);
}

extern "C" int lap_kemeny(lap_graph *g, int32_t root, int64_t omega, uint64_t seed, double *kappa, double *se,
                          void *hip_stream) {
    lap_sample_args a = default_args(root, omega, seed, 1);
    lap_estimates e;
    std::memset(&e, 0, sizeof e);
    e.kemeny = kappa;
    e.kemeny_se = se;
    if (!kappa && !se) return fail(LAP_EINVAL, "no output requested");
    return lap_estimate(g, &a, &e, hip_stream);
}
