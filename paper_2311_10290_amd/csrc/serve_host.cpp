// Serving loop over one resident graph (lap_server_*): queries are queued,
// admitted while their result regions fit in a device arena, cut into work
// items and batched -- one item per active query per round, so short queries
// are not stuck behind long ones -- into launches that run concurrently on
// several streams.  New queries join the next launch while earlier launches
// are still on the device (continuous batching).  Completed queries are
// assembled on the host in FP64 in a fixed order.
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <deque>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "lap_host.h"
#include "lap_launch.h"
#include "serve_arena.h"

using namespace lap;

namespace {

struct SQuery {
    lap_query q;
    int64_t off = -1, words = 0;
    int64_t n_items = 0, issued = 0, finished = 0;
    int64_t next_wilson = 0, next_pi = 0, next_walk = 0;
    double t_submit = 0, t_start = -1;
    int status = LAP_OK;
    bool cancelled = false;     // no new items; dropped once its issued items are back
};

struct SLaunch {
    hipStream_t s = nullptr;
    hipEvent_t ev = nullptr;
    bool busy = false;
    ServeItem *h_items = nullptr;   // pinned host copy of the item table
    DevBuf d_items, counter, err;
    std::vector<int64_t> serials;   // query of each item
    int64_t n_items = 0;
};

double now_s(std::chrono::steady_clock::time_point t0) {
    return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
}

int64_t result_words(const lap_query &q) { return (q.kind == LAP_Q_RESISTANCE ? 4 : 2) * q.budget; }

int64_t item_count(const lap_query &q, int32_t chunk) {
    const int64_t tiles = (q.budget + 63) / 64;
    if (q.kind == LAP_Q_KEMENY) return (q.budget + chunk - 1) / chunk + tiles;
    return tiles;
}

}  // namespace

struct lap_server {
    lap_graph *g = nullptr;
    lap_server_config cfg{};
    int64_t n = 0;
    DevBuf arena, state, epoch, stats;
    std::vector<SLaunch> launches;
    std::map<int64_t, SQuery> active;     // by serial
    std::deque<SQuery> queue;
    std::vector<lap_query_result> done;
    WordArena words;                      // free runs of the result arena
    std::mutex mu;
    double tr_lv = 0, s_lv = 0;
    int64_t serial = 0;
    uint64_t k1 = 0;
    uint64_t deadline = 0;
    std::chrono::steady_clock::time_point t0;
    ~lap_server() {
        for (auto &L : launches) {
            if (L.s) (void)hipStreamSynchronize(L.s);
            if (L.ev) (void)hipEventDestroy(L.ev);
            if (L.s) (void)hipStreamDestroy(L.s);
            if (L.h_items) (void)hipHostFree(L.h_items);
            L.d_items.release();
            L.counter.release();
            L.err.release();
        }
        arena.release();
        state.release();
        epoch.release();
        stats.release();
    }
};

namespace {

// a result record for a query that ends without a value
lap_query_result ended(const lap_server *s, const SQuery &Q, int status) {
    lap_query_result r;
    std::memset(&r, 0, sizeof r);
    r.qid = Q.q.qid;
    r.kind = Q.q.kind;
    r.status = status;
    r.value = r.se = NAN;
    r.t_submit = Q.t_submit;
    r.t_start = Q.t_start;
    r.t_done = now_s(s->t0);
    return r;
}

double degree(const lap_graph *g, int32_t u) { return (double)(g->csr.rp[u + 1] - g->csr.rp[u]); }

// FP64 assembly of a finished query from its result words (fixed order)
void assemble(lap_server *s, const SQuery &Q, const std::vector<uint64_t> &w, lap_query_result &r) {
    const int64_t b = Q.q.budget;
    const double nn = (double)s->n;
    std::vector<double> z((size_t)b);
    if (Q.q.kind == LAP_Q_KEMENY) {
        long long tot = 0;
        for (int64_t i = 0; i < b; ++i) tot += (long long)((int64_t)w[i] - (int64_t)w[b + i]);
        const double mean = (double)tot / (double)b;
        double sq = 0;
        for (int64_t i = 0; i < b; ++i) {
            const double d = (double)((int64_t)w[i] - (int64_t)w[b + i]) - mean;
            sq += d * d;
        }
        r.value = mean;
        r.se = b > 1 ? std::sqrt(sq / (double)(b - 1)) / std::sqrt((double)b) : NAN;
        return;
    }
    if (Q.q.kind == LAP_Q_CLOSENESS) {
        const double du = degree(s->g, Q.q.u);
        for (int64_t i = 0; i < b; ++i) {
            double nl;
            std::memcpy(&nl, &w[b + i], sizeof nl);
            z[i] = (double)(int64_t)w[i] / du - 2.0 * nl / nn;
        }
    } else {
        const double ds = degree(s->g, Q.q.u), dt = degree(s->g, Q.q.w);
        for (int64_t i = 0; i < b; ++i)
            z[i] = (double)(int64_t)w[i] / ds - (double)(int64_t)w[b + i] / dt + (double)(int64_t)w[2 * b + i] / dt -
                   (double)(int64_t)w[3 * b + i] / ds;
    }
    double sum = 0;
    for (int64_t i = 0; i < b; ++i) sum += z[i];
    const double mean = sum / (double)b;
    double sq = 0;
    for (int64_t i = 0; i < b; ++i) sq += (z[i] - mean) * (z[i] - mean);
    const double se = b > 1 ? std::sqrt(sq / (double)(b - 1)) / std::sqrt((double)b) : NAN;
    if (Q.q.kind == LAP_Q_RESISTANCE) {
        r.value = mean;
        r.se = se;
        return;
    }
    // closeness: L^dagger_uu from the element-wise equation, Tr L^dagger = Tr L_v^{-1} - S/n
    const double ld = mean + s->s_lv / (nn * nn);
    const double tr = s->tr_lv - s->s_lv / nn;
    const double den = tr + nn * ld;
    r.value = (nn - 1.0) / den;
    r.se = std::fabs((nn - 1.0) * nn / (den * den)) * se;
}

int retire(lap_server *s, SLaunch &L) {
    DevErr e{0, 0};
    HIP_TRY(hipMemcpy(&e, L.err.ptr, sizeof e, hipMemcpyDeviceToHost));
    for (int64_t sr : L.serials) {
        auto it = s->active.find(sr);
        if (it == s->active.end()) continue;
        it->second.finished += 1;
        if (e.code != kErrNone) it->second.status = LAP_ERANGE;
    }
    L.busy = false;
    L.serials.clear();
    // finalise every query whose items have all come back (a cancelled one:
    // every item it had issued)
    std::vector<int64_t> fin;
    for (auto &kv : s->active)
        if (kv.second.finished == (kv.second.cancelled ? kv.second.issued : kv.second.n_items)) fin.push_back(kv.first);
    for (int64_t sr : fin) {
        SQuery &Q = s->active[sr];
        if (Q.cancelled) {
            s->done.push_back(ended(s, Q, LAP_ECANCELED));
            s->words.release(Q.off, Q.words);
            s->active.erase(sr);
            continue;
        }
        lap_query_result r;
        std::memset(&r, 0, sizeof r);
        r.qid = Q.q.qid;
        r.kind = Q.q.kind;
        r.status = Q.status;
        r.t_submit = Q.t_submit;
        r.t_start = Q.t_start;
        if (Q.status == LAP_OK) {
            std::vector<uint64_t> w((size_t)Q.words);
            HIP_TRY(hipMemcpy(w.data(), s->arena.as<uint64_t>() + Q.off, 8 * Q.words, hipMemcpyDeviceToHost));
            assemble(s, Q, w, r);
        } else {
            r.value = r.se = NAN;
        }
        r.t_done = now_s(s->t0);
        s->done.push_back(r);
        s->words.release(Q.off, Q.words);
        s->active.erase(sr);
    }
    if (e.code != kErrNone) {
        // an abandoned sample leaves walk state behind: clear every slot
        const int64_t slots = (int64_t)s->cfg.launches * s->cfg.waves;
        for (auto &O : s->launches)
            if (O.busy) HIP_TRY(hipStreamSynchronize(O.s));
        HIP_TRY(launch_fill_u64(s->state.as<uint64_t>(), 0, slots * s->n, L.s));
        HIP_TRY(launch_fill_u64(s->epoch.as<uint64_t>(), 0, slots / 2 + 1, L.s));
        HIP_TRY(hipStreamSynchronize(L.s));
        return fail(LAP_ERANGE, "serving kernel stopped (time limit or inconsistent state)");
    }
    return LAP_OK;
}

// next work item of a query for a launch of class cls (0: walk tiles, 1:
// Wilson samples, 2: either), or false if it has none left of that class
bool next_item(lap_server *s, SQuery &Q, ServeItem &it, int cls) {
    if (Q.cancelled) return false;
    const int64_t b = Q.q.budget;
    std::memset(&it, 0, sizeof it);
    it.budget = b;
    it.qid = Q.q.qid;
    it.u = Q.q.u;
    it.w = Q.q.w;
    it.out_off = Q.off;
    if (Q.q.kind == LAP_Q_KEMENY) {
        const bool wil_left = Q.next_wilson < b && cls != 0;
        const bool pi_left = Q.next_pi < b && cls != 1;
        if (!wil_left && !pi_left) return false;
        if (wil_left && (!pi_left || Q.issued % 2 == 0)) {
            it.kind = 0;
            it.first = Q.next_wilson;
            it.count = (int32_t)std::min<int64_t>(s->cfg.wilson_chunk, b - Q.next_wilson);
            Q.next_wilson += it.count;
        } else {
            it.kind = 2;
            it.first = Q.next_pi;
            it.count = (int32_t)std::min<int64_t>(64, b - Q.next_pi);
            Q.next_pi += it.count;
        }
    } else {
        if (cls == 1 || Q.next_walk >= b) return false;
        it.kind = Q.q.kind == LAP_Q_CLOSENESS ? 3 : 4;
        it.first = Q.next_walk;
        it.count = (int32_t)std::min<int64_t>(64, b - Q.next_walk);
        Q.next_walk += it.count;
    }
    Q.issued += 1;
    return true;
}

// With two or more launches, even-numbered streams run walk tiles and odd
// ones Wilson samples, so short walk queries never wait for a Wilson sample
// of a Kemeny query that shares their launch.
int launch(lap_server *s, int idx) {
    SLaunch &L = s->launches[idx];
    const int cls = s->launches.size() < 2 ? 2 : (idx % 2);
    int64_t cnt = 0;
    const double t = now_s(s->t0);
    if (cls == 1) {
        // Wilson launches: at most one sample per state slot, oldest query
        // first, so that a launch lasts about one sample and the samples of a
        // Kemeny query finish together in as few launches as possible
        const int64_t cap = std::min<int64_t>({(int64_t)s->cfg.items_per_launch, (int64_t)s->cfg.waves,
                                               (int64_t)s->cfg.wilson_slots});
        for (auto &kv : s->active) {
            SQuery &Q = kv.second;
            while (cnt < cap && Q.issued < Q.n_items && next_item(s, Q, L.h_items[cnt], cls)) {
                L.serials.push_back(kv.first);
                if (Q.t_start < 0) Q.t_start = t;
                ++cnt;
            }
            if (cnt >= cap) break;
        }
    }
    bool any = cls != 1;
    while (any && cnt < s->cfg.items_per_launch) {
        any = false;
        for (auto &kv : s->active) {
            SQuery &Q = kv.second;
            if (cnt >= s->cfg.items_per_launch) break;
            if (Q.issued >= Q.n_items) continue;
            if (next_item(s, Q, L.h_items[cnt], cls)) {
                L.serials.push_back(kv.first);
                if (Q.t_start < 0) Q.t_start = t;
                ++cnt;
                any = true;
            }
        }
    }
    if (cnt == 0) return LAP_OK;
    L.n_items = cnt;
    HIP_TRY(hipMemcpyAsync(L.d_items.ptr, L.h_items, sizeof(ServeItem) * cnt, hipMemcpyHostToDevice, L.s));
    HIP_TRY(launch_fill_u64(L.counter.as<uint64_t>(), 0, 1, L.s));
    HIP_TRY(launch_fill_u64(L.err.as<uint64_t>(), 0, 1, L.s));
    ServeParams p;
    std::memset(&p, 0, sizeof p);
    lap_graph *g = s->g;
    p.n = s->n;
    p.nnz = g->csr.rp[s->n];
    p.nbr = g->nbr.as<uint64_t>();
    p.col = g->col.as<int32_t>();
    p.arcs = (const ulonglong2 *)g->arcs.ptr;
    p.root = s->cfg.root;
    p.k0 = s->cfg.seed;
    p.k1 = s->k1;
    p.items = L.d_items.as<ServeItem>();
    p.n_items = cnt;
    p.counter = L.counter.as<unsigned long long>();
    p.state = s->state.as<uint64_t>();
    p.slot_epoch = s->epoch.as<uint32_t>();
    p.slot_base = (int64_t)idx * s->cfg.waves;
    p.arena = s->arena.as<uint64_t>();
    p.stats = s->stats.as<unsigned long long>();
    p.err = L.err.as<DevErr>();
    p.deadline = s->deadline;
    if (cls == 1 && s->cfg.wilson_group > 1) {
        // a Wilson-only launch: W wavefronts per sample, one workgroup per state
        // slot of the launch
        HIP_TRY(launch_serve_group(p, s->cfg.wilson_group, std::min<int64_t>(s->cfg.waves, cnt), L.s));
    } else {
        HIP_TRY(launch_serve(p, std::min<int64_t>(s->cfg.waves, cnt), L.s));
    }
    HIP_TRY(hipEventRecord(L.ev, L.s));
    L.busy = true;
    return LAP_OK;
}

}  // namespace

extern "C" int lap_server_create(lap_graph *g, const lap_server_config *cfg, void *hip_stream, lap_server **out) {
    if (!g || !out) return fail(LAP_EINVAL, "graph or output is NULL");
    lap_server *s = new (std::nothrow) lap_server();
    if (!s) return fail(LAP_ENOMEM, "host allocation failed");
    s->g = g;
    s->n = g->csr.n;
    if (cfg) s->cfg = *cfg;
    lap_server_config &c = s->cfg;
    if (c.root < -1 || c.root >= s->n || c.global_samples < 0 || c.arena_bytes < 0 || c.launches < 0 ||
        c.waves < 0 || c.items_per_launch < 0 || c.wilson_chunk < 0 || c.wilson_slots < 0 ||
        (c.wilson_group != 0 && c.wilson_group != 1 && c.wilson_group != 2 && c.wilson_group != 4 &&
         c.wilson_group != 8)) {
        delete s;
        return fail(LAP_EINVAL, "bad server configuration");
    }
    if (c.root < 0) c.root = g->max_deg_node;
    if (c.global_samples == 0) c.global_samples = 256;
    if (c.arena_bytes == 0) c.arena_bytes = (int64_t)64 << 20;
    if (c.launches == 0) c.launches = 5;
    if (c.waves == 0) c.waves = 4 * g->n_cu;
    if (c.items_per_launch == 0) c.items_per_launch = 4096;
    if (c.wilson_chunk == 0) c.wilson_chunk = 1;
    if (c.timeout_s <= 0) c.timeout_s = 300.0;
    if (c.wilson_group == 0) c.wilson_group = s->n >= (1 << 16) ? 4 : 1;
    if (c.wilson_slots == 0 || c.wilson_slots > c.waves) c.wilson_slots = c.waves;
    s->k1 = ((uint64_t)c.stream << 32) | (uint64_t)(uint32_t)c.root;
    s->deadline = (uint64_t)(c.timeout_s * g->clock_khz * 1000.0);
    // cached global terms: Tr(L_v^{-1}) and 1^T L_v^{-1} 1 from one Wilson +
    // uniform-walk run keyed by a reserved query id
    {
        lap_sample_args a;
        std::memset(&a, 0, sizeof a);
        a.n_samples = c.global_samples;
        a.seed = c.seed;
        a.root = c.root;
        a.stream = c.stream;
        a.qid = LAP_SERVER_GLOBAL_QID;
        a.want = LAP_WANT_Y1 | LAP_WANT_Y2_UNIFORM;
        a.n_blocks = 1;
        a.timeout_s = c.timeout_s;
        std::vector<int64_t> y1((size_t)s->n), y2((size_t)s->n);
        lap_counts cn;
        std::memset(&cn, 0, sizeof cn);
        cn.y1 = y1.data();
        cn.y2 = y2.data();
        int rc = lap_sample_forests(g, &a, &cn, hip_stream);
        if (rc != LAP_OK) {
            delete s;
            return rc;
        }
        double t1 = 0, t2 = 0;
        for (int64_t u = 0; u < s->n; ++u) {
            if (u == c.root) continue;
            const double du = degree(g, (int32_t)u);
            t1 += (double)y1[u] / ((double)c.global_samples * du);
            t2 += (double)y2[u] / ((double)c.global_samples * du);
        }
        s->tr_lv = t1;
        s->s_lv = (double)s->n * t2;
    }
    const int64_t words = c.arena_bytes / 8;
    const int64_t slots = (int64_t)c.launches * c.waves;
    if (s->arena.ensure(8 * (size_t)words) || s->state.ensure(8 * (size_t)slots * (size_t)s->n) ||
        s->epoch.ensure(8 * (size_t)(slots / 2 + 1)) || s->stats.ensure(8 * kNumStats)) {
        delete s;
        return fail(LAP_ENOMEM, "cannot allocate serving memory");
    }
    hipStream_t hs = (hipStream_t)hip_stream;
    if (launch_fill_u64(s->state.as<uint64_t>(), 0, slots * s->n, hs) != hipSuccess ||
        launch_fill_u64(s->epoch.as<uint64_t>(), 0, slots / 2 + 1, hs) != hipSuccess ||
        launch_fill_u64(s->stats.as<uint64_t>(), 0, kNumStats, hs) != hipSuccess || hipStreamSynchronize(hs) != hipSuccess) {
        delete s;
        return fail(LAP_EDEVICE, "cannot clear serving memory");
    }
    s->words.reset(words);
    s->launches.resize((size_t)c.launches);
    for (auto &L : s->launches) {
        if (hipStreamCreateWithFlags(&L.s, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&L.ev, hipEventDisableTiming) != hipSuccess ||
            hipHostMalloc((void **)&L.h_items, sizeof(ServeItem) * c.items_per_launch, hipHostMallocDefault) != hipSuccess ||
            L.d_items.ensure(sizeof(ServeItem) * c.items_per_launch) || L.counter.ensure(8) || L.err.ensure(8)) {
            delete s;
            return fail(LAP_ENOMEM, "cannot create serving streams");
        }
    }
    s->t0 = std::chrono::steady_clock::now();
    *out = s;
    return LAP_OK;
}

extern "C" int lap_server_submit(lap_server *s, const lap_query *q) {
    if (!s || !q) return fail(LAP_EINVAL, "server or query is NULL");
    if (q->kind < LAP_Q_CLOSENESS || q->kind > LAP_Q_KEMENY || q->budget < 1 || q->qid < 0 ||
        (uint64_t)q->qid == LAP_SERVER_GLOBAL_QID)
        return fail(LAP_EINVAL, "bad query kind, budget or id");
    if (q->kind != LAP_Q_KEMENY && (q->u < 0 || q->u >= s->n))
        return fail(LAP_EINVAL, "query node out of range");
    if (q->kind == LAP_Q_RESISTANCE && (q->w < 0 || q->w >= s->n))
        return fail(LAP_EINVAL, "query node out of range");
    if (8 * result_words(*q) > s->cfg.arena_bytes) return fail(LAP_ENOMEM, "query larger than the result arena");
    std::lock_guard<std::mutex> lk(s->mu);
    SQuery Q;
    Q.q = *q;
    Q.words = result_words(*q);
    Q.n_items = item_count(*q, s->cfg.wilson_chunk);
    Q.t_submit = now_s(s->t0);
    s->queue.push_back(Q);
    return LAP_OK;
}

extern "C" int lap_server_step(lap_server *s, int32_t wait) {
    if (!s) return fail(LAP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    // 1. retire launches that have completed (with wait: the oldest busy one)
    int rc = LAP_OK;
    bool retired = false;
    for (auto &L : s->launches) {
        if (!L.busy) continue;
        const hipError_t q = hipEventQuery(L.ev);
        if (q == hipSuccess) {
            int r2 = retire(s, L);
            if (r2 != LAP_OK) rc = r2;
            retired = true;
        } else if (q != hipErrorNotReady) {
            return fail(LAP_EDEVICE, std::string("serving launch failed: ") + hipGetErrorString(q));
        }
    }
    if (wait && !retired) {
        for (auto &L : s->launches)
            if (L.busy) {
                HIP_TRY(hipEventSynchronize(L.ev));
                int r2 = retire(s, L);
                if (r2 != LAP_OK) rc = r2;
                break;
            }
    }
    // 2. admit queued queries while their result regions fit in the arena
    while (!s->queue.empty()) {
        SQuery &Q = s->queue.front();
        const int64_t off = s->words.alloc(Q.words);
        if (off < 0) break;
        Q.off = off;
        s->active[s->serial++] = Q;
        s->queue.pop_front();
    }
    // 3. start launches on idle streams with the active queries' next items
    for (size_t i = 0; i < s->launches.size(); ++i)
        if (!s->launches[i].busy) {
            int r2 = launch(s, (int)i);
            if (r2 != LAP_OK) return r2;
        }
    return rc;
}

extern "C" int lap_server_cancel(lap_server *s, int64_t qid) {
    if (!s) return fail(LAP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    for (auto it = s->queue.begin(); it != s->queue.end(); ++it)
        if (it->q.qid == qid) {
            s->done.push_back(ended(s, *it, LAP_ECANCELED));
            s->queue.erase(it);
            return LAP_OK;
        }
    for (auto it = s->active.begin(); it != s->active.end(); ++it) {
        SQuery &Q = it->second;
        if (Q.q.qid != qid || Q.cancelled) continue;
        Q.cancelled = true;
        if (Q.finished == Q.issued) {
            // nothing of it on the device: its arena region is free at once
            s->done.push_back(ended(s, Q, LAP_ECANCELED));
            s->words.release(Q.off, Q.words);
            s->active.erase(it);
        }
        return LAP_OK;
    }
    return fail(LAP_EINVAL, "no queued or running query with id " + std::to_string(qid));
}

extern "C" int lap_server_poll(lap_server *s, lap_query_result *out, int32_t max, int32_t *n_out) {
    if (!s || (!out && max > 0) || !n_out) return fail(LAP_EINVAL, "bad poll arguments");
    std::lock_guard<std::mutex> lk(s->mu);
    const int32_t k = (int32_t)std::min<size_t>((size_t)std::max(max, 0), s->done.size());
    for (int32_t i = 0; i < k; ++i) out[i] = s->done[i];
    s->done.erase(s->done.begin(), s->done.begin() + k);
    *n_out = k;
    return LAP_OK;
}

extern "C" int lap_server_pending(lap_server *s, int64_t *queued, int64_t *active, int64_t *inflight) {
    if (!s) return fail(LAP_EINVAL, "server is NULL");
    std::lock_guard<std::mutex> lk(s->mu);
    if (queued) *queued = (int64_t)s->queue.size();
    if (active) *active = (int64_t)s->active.size();
    int64_t f = 0;
    for (auto &L : s->launches) f += L.busy;
    if (inflight) *inflight = f;
    return LAP_OK;
}

extern "C" int lap_server_globals(const lap_server *s, double *trace_lv, double *sum_lv) {
    if (!s) return fail(LAP_EINVAL, "server is NULL");
    if (trace_lv) *trace_lv = s->tr_lv;
    if (sum_lv) *sum_lv = s->s_lv;
    return LAP_OK;
}

extern "C" void lap_server_free(lap_server *s) { delete s; }
