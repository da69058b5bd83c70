// Many independent estimation jobs (graph, landmark, sample budget) in one
// persistent launch.  Every job is the same computation as one lap_estimate
// call (Wilson samples, uniform- and stationary-start absorbed walks, FP64
// assembly; Alg. 2 and Alg. 4) and draws the same Philox stream, so each
// job's counts equal those of the plain path bit for bit.
//
// Work items, fetched by resident wavefronts from one atomic counter:
//   kind 0  a chunk of consecutive Wilson samples of one job, sized so that
//           samples * nodes is about the tuning's chunk_nodes; the wave clears
//           its state slot for the job's node range, then runs the samples
//           with the wave-cooperative sampler;
//   kind 1  64 uniform-start absorbed walks of one job, one per lane;
//   kind 2  64 stationary-start absorbed walks of one job.
// Items come job by job, largest graphs first (Wilson chunks, then walk
// tiles), so the waves in flight share a few graphs and short items fill the
// tail.
#include "lap_device.h"
#include "lap_launch.h"
#include "walks.h"
#include "wave_sample.h"

namespace lap {

__global__ __launch_bounds__(64) void batch_kernel(BatchParams p) {
    __shared__ WaveShared sh;
    __shared__ int64_t item_sh;
    const int lane = (int)threadIdx.x;
    uint64_t *st = p.state + (int64_t)blockIdx.x * p.max_n;
    const uint64_t t0 = wall_clock64();
    WaveStats ws;
    unsigned long long walk_steps = 0;
    while (true) {
        if (lane == 0) item_sh = err_set(p.err) ? p.n_items : (int64_t)atomicAdd(p.counter, 1ull);
        __syncthreads();
        const int64_t it = item_sh;
        __syncthreads();
        if (it >= p.n_items) break;
        const BatchItem bi = p.items[it];
        const BatchJobDev jb = p.jobs[bi.job];
        const uint64_t *nbr = p.nbr + jb.node_off;
        const int32_t *col = p.col + jb.col_off;
        if (bi.kind == 0) {
            for (int64_t i = lane; i < jb.n; i += 64) st[i] = 0ull;
            __syncthreads();
            WaveSampleArgs c;
            c.n = jb.n;
            c.nnz = jb.nnz;
            c.nbr = nbr;
            c.col = col;
            c.root = jb.root;
            c.k0 = jb.k0;
            c.k1 = jb.k1;
            c.qid = jb.qid;
            c.st = st;
            c.y1b = p.y1 ? p.y1 + jb.node_off : nullptr;
            c.keep_next = nullptr;
            c.keep_draws = nullptr;
            c.err = p.err;
            c.t0 = t0;
            c.deadline = p.deadline;
            c.scan_offset = 0;
            uint32_t ep = 0;
            bool ok = true;
            for (int64_t s = bi.first; s < bi.first + bi.count && ok; ++s) {
                ep ^= 1u;
                c.sample = s;
                c.ep = ep;
                int64_t y1 = 0;
                ok = wave_wilson_sample(c, sh, &y1, ws);
                if (ok && lane == 0) {
                    p.y1s[jb.sample_off + s] = y1;
                    ++ws.trees;
                }
            }
            if (!ok) break;
        } else {
            const WalkGraph g{nbr, col, nullptr, jb.n, jb.nnz, jb.root, jb.k0, jb.k1, jb.qid};
            const int64_t i = bi.first + lane;
            if (lane < bi.count) {
                unsigned long long *y2 = bi.kind == 1 ? p.y2 + jb.node_off : nullptr;
                const int64_t len = absorbed_walk(g, (uint32_t)bi.kind, i, y2, p.err, t0, p.deadline);
                if (len >= 0) {
                    (bi.kind == 1 ? p.len_u : p.len_p)[jb.sample_off + i] = len;
                    walk_steps += (unsigned long long)len;
                }
            }
        }
    }
    flush_wave_stats(ws, p.stats);
    const int64_t wsum = wave_sum_i64((int64_t)walk_steps);
    if (lane == 0) atomicAdd(&p.stats[kStatAbsorbed], (unsigned long long)wsum);
}

hipError_t launch_batch(const BatchParams &p, int64_t waves, hipStream_t s) {
    hipLaunchKernelGGL(batch_kernel, dim3((unsigned)waves), dim3(64), 0, s, p);
    return hipGetLastError();
}

// --------------------------------------------------------------- assembly
// One workgroup per job: S = sum_w Y2[w]/d_w, diag_u, Tr, c_u, and Kemeny's
// constant with its standard error from the per-sample arrays (fixed-order
// reductions).
constexpr int kBA = 256;

__device__ double bsum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBA / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

__device__ long long bsum_ll(long long v, long long *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kBA / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const long long r = sh[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(kBA) void batch_assemble_kernel(BatchParams p) {
    __shared__ double shd[kBA];
    __shared__ long long shl[kBA];
    const BatchJobDev jb = p.jobs[blockIdx.x];
    const uint64_t *nbr = p.nbr + jb.node_off;
    unsigned long long *y1 = p.y1 + jb.node_off;
    const unsigned long long *y2 = p.y2 + jb.node_off;
    double *diag = p.diag + jb.node_off, *clo = p.closeness + jb.node_off;
    const double om = (double)jb.omega, nn = (double)jb.n;
    double acc = 0.0;
    for (int64_t w = threadIdx.x; w < jb.n; w += kBA)
        if (w != jb.root) acc += (double)y2[w] / (double)nbr_deg(nbr[w]);
    const double S = bsum(acc, shd);
    double tr = 0.0;
    for (int64_t u = threadIdx.x; u < jb.n; u += kBA) {
        double d = S / (om * nn);
        if (u != jb.root) {
            // the kernel counted draws beyond the first; restore the baseline
            const unsigned long long full = y1[u] + (unsigned long long)jb.omega;
            y1[u] = full;
            d += ((double)full - 2.0 * (double)y2[u]) / (om * (double)nbr_deg(nbr[u]));
        }
        diag[u] = d;
        tr += d;
    }
    const double Tr = bsum(tr, shd);
    for (int64_t u = threadIdx.x; u < jb.n; u += kBA)
        clo[u] = jb.n > 1 ? (nn - 1.0) / (Tr + nn * diag[u]) : 0.0;
    const int64_t *ys = p.y1s + jb.sample_off, *lp = p.len_p + jb.sample_off;
    long long zs = 0;
    for (int64_t i = threadIdx.x; i < jb.omega; i += kBA) zs += (long long)(ys[i] - lp[i]);
    const long long Z = bsum_ll(zs, shl);
    const double mean = (double)Z / om;
    double sq = 0.0;
    for (int64_t i = threadIdx.x; i < jb.omega; i += kBA) {
        const double dz = (double)(ys[i] - lp[i]) - mean;
        sq += dz * dz;
    }
    const double SQ = bsum(sq, shd);
    if (threadIdx.x == 0) {
        p.trace[blockIdx.x] = Tr;
        p.kemeny[blockIdx.x] = mean;
        p.kemeny_se[blockIdx.x] = jb.omega > 1 ? sqrt(SQ / (om - 1.0)) / sqrt(om) : __builtin_nan("");
    }
}

hipError_t launch_batch_assemble(const BatchParams &p, int32_t n_jobs, hipStream_t s) {
    hipLaunchKernelGGL(batch_assemble_kernel, dim3((unsigned)n_jobs), dim3(kBA), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
