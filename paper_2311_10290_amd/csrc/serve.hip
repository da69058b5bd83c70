// Query execution for the serving loop: one launch runs a list of work items
// drawn from several queries; resident wavefronts take items from an atomic
// counter (as in the batched kernel).  Items:
//   kind 0  consecutive Wilson samples of a Kemeny query (wave-cooperative)
//   kind 2  64 stationary-start absorbed walks of a Kemeny query
//   kind 3  64 walks from node u of a closeness query
//   kind 4  64 walk pairs (from s and from t) of a resistance query
// Each query's random stream is keyed by its id (counter word 3), and every
// result is written at a fixed place in the query's region of the result
// arena, so a query's result does not depend on what it was batched with.
#include "lap_device.h"
#include "lap_launch.h"
#include "walks.h"
#include "group_sample.h"
#include "wave_sample.h"

namespace lap {

__global__ __launch_bounds__(64) void serve_kernel(ServeParams p) {
    __shared__ WaveShared sh;
    __shared__ int64_t item_sh;
    const int lane = (int)threadIdx.x;
    const int64_t slot = p.slot_base + blockIdx.x;
    uint64_t *st = p.state + slot * p.n;
    uint32_t ep = p.slot_epoch[slot];
    const uint64_t t0 = wall_clock64();
    WaveStats ws;
    unsigned long long walk_steps = 0;
    while (true) {
        if (lane == 0) item_sh = err_set(p.err) ? p.n_items : (int64_t)atomicAdd(p.counter, 1ull);
        __syncthreads();
        const int64_t it = item_sh;
        __syncthreads();
        if (it >= p.n_items) break;
        const ServeItem q = p.items[it];
        uint64_t *out = p.arena + q.out_off;
        const WalkGraph g{p.nbr, p.col, p.arcs, p.n, p.nnz, p.root, p.k0, p.k1, (uint64_t)q.qid};
        if (q.kind == 0) {
            WaveSampleArgs c;
            c.n = p.n;
            c.nnz = p.nnz;
            c.nbr = p.nbr;
            c.col = p.col;
            c.root = p.root;
            c.k0 = p.k0;
            c.k1 = p.k1;
            c.qid = (uint64_t)q.qid;
            c.st = st;
            c.y1b = nullptr;
            c.keep_next = nullptr;
            c.keep_draws = nullptr;
            c.err = p.err;
            c.t0 = t0;
            c.deadline = p.deadline;
            c.scan_offset = 0;
            bool ok = true;
            for (int64_t s = q.first; s < q.first + q.count && ok; ++s) {
                ep ^= 1u;
                c.sample = s;
                c.ep = ep;
                int64_t y1 = 0;
                ok = wave_wilson_sample(c, sh, &y1, ws);
                if (ok && lane == 0) {
                    out[s] = (uint64_t)y1;
                    ++ws.trees;
                }
            }
            if (!ok) break;
        } else if (lane < q.count) {
            const int64_t i = q.first + lane;
            if (q.kind == 2) {
                const int64_t len = absorbed_walk(g, 2, i, nullptr, p.err, t0, p.deadline);
                if (len >= 0) {
                    out[q.budget + i] = (uint64_t)len;
                    walk_steps += (unsigned long long)len;
                }
            } else if (q.kind == 3) {
                int64_t da = 0, db = 0;
                double nl = 0.0;
                if (query_walk(g, q.u, 0, i, q.u, q.u, &da, &db, &nl, p.err, t0, p.deadline)) {
                    out[i] = (uint64_t)da;
                    out[q.budget + i] = __double_as_longlong(nl);
                }
            } else if (q.kind == 4) {
                int64_t ss = 0, st_ = 0, tt = 0, ts = 0;
                double nl = 0.0;
                if (query_walk(g, q.u, 0, i, q.u, q.w, &ss, &st_, &nl, p.err, t0, p.deadline) &&
                    query_walk(g, q.w, 1, i, q.w, q.u, &tt, &ts, &nl, p.err, t0, p.deadline)) {
                    out[i] = (uint64_t)ss;
                    out[q.budget + i] = (uint64_t)st_;
                    out[2 * q.budget + i] = (uint64_t)tt;
                    out[3 * q.budget + i] = (uint64_t)ts;
                }
            }
        }
    }
    if (lane == 0) p.slot_epoch[slot] = ep;
    flush_wave_stats(ws, p.stats);
    const int64_t wsum = wave_sum_i64((int64_t)walk_steps);
    if (lane == 0) atomicAdd(&p.stats[kStatAbsorbed], (unsigned long long)wsum);
}

// Wilson-only launches with W wavefronts per sample (group_sample.h): one
// workgroup per state slot pulls kind-0 items; any other kind is skipped (the
// host never puts one in such a launch).
template <int W>
__global__ __launch_bounds__(kWave * W, 4) void serve_group_kernel(ServeParams p) {
    __shared__ GroupShared<W> sh;
    __shared__ int64_t item_sh;
    const int tid = (int)threadIdx.x;
    const int64_t slot = p.slot_base + blockIdx.x;
    uint64_t *st = p.state + slot * p.n;
    uint32_t ep = p.slot_epoch[slot];
    const uint64_t t0 = wall_clock64();
    WaveStats ws;
    while (true) {
        if (tid == 0) item_sh = err_set(p.err) ? p.n_items : (int64_t)atomicAdd(p.counter, 1ull);
        __syncthreads();
        const int64_t it = item_sh;
        __syncthreads();
        if (it >= p.n_items) break;
        const ServeItem q = p.items[it];
        if (q.kind != 0) continue;
        uint64_t *out = p.arena + q.out_off;
        WaveSampleArgs c;
        c.n = p.n;
        c.nnz = p.nnz;
        c.nbr = p.nbr;
        c.col = p.col;
        c.root = p.root;
        c.k0 = p.k0;
        c.k1 = p.k1;
        c.qid = (uint64_t)q.qid;
        c.st = st;
        c.y1b = nullptr;
        c.keep_next = nullptr;
        c.keep_draws = nullptr;
        c.err = p.err;
        c.t0 = t0;
        c.deadline = p.deadline;
        c.scan_offset = 0;
        bool ok = true;
        for (int64_t s = q.first; s < q.first + q.count && ok; ++s) {
            ep ^= 1u;
            c.sample = s;
            c.ep = ep;
            int64_t y1 = 0;
            ok = group_wilson_sample<W>(c, sh, &y1, ws);
            if (ok && tid == 0) {
                out[s] = (uint64_t)y1;
                ++ws.trees;
            }
        }
        if (!ok) break;
    }
    if (tid == 0) p.slot_epoch[slot] = ep;
    flush_group_stats(ws, p.stats);
}

hipError_t launch_serve_group(const ServeParams &p, int waves, int64_t groups, hipStream_t s) {
    switch (waves) {
    case 2:
        hipLaunchKernelGGL(serve_group_kernel<2>, dim3((unsigned)groups), dim3(kWave * 2), 0, s, p);
        break;
    case 4:
        hipLaunchKernelGGL(serve_group_kernel<4>, dim3((unsigned)groups), dim3(kWave * 4), 0, s, p);
        break;
    case 8:
        hipLaunchKernelGGL(serve_group_kernel<8>, dim3((unsigned)groups), dim3(kWave * 8), 0, s, p);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_serve(const ServeParams &p, int64_t waves, hipStream_t s) {
    hipLaunchKernelGGL(serve_kernel, dim3((unsigned)waves), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
