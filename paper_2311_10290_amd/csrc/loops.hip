// Loop-included paths of the Wilson stacks (Sec. 3.4): after a Wilson launch
// with at most one sample per slot, path i starts where absorbed walk i of the
// given kind starts and follows the bottom entries of sample i's stacks --
// at its c-th departure from u it takes stack entry S_i[u][c], the same
// Philox draw (i, u, c, qid) the sampler used -- until it reaches v.  By the
// loop-erased-walk lemma of Sec. 3.4 the path is distributed as a v-absorbed
// walk from its start, so its departures estimate what Alg. 2's and Alg. 4's
// walks estimate, with no draws of their own.
//
// One lane per path; each path counts its departures per node in its slot's
// counter array (cleared before the launch).  Every entry a path uses was
// drawn by the sample (popped, or the tree edge on top), so c < k_u always
// holds; a violation stops the kernel as an inconsistency.
#include "lap_device.h"
#include "lap_launch.h"

namespace lap {

__global__ __launch_bounds__(64) void loop_included_kernel(LoopParams p) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (slot >= p.n_paths) return;
    const int64_t n = p.n;
    const int64_t i = p.sample_begin + slot;
    const uint64_t *st = p.state + slot * n;
    int32_t *cnt = p.cnt + slot * n;
    const uint32_t ep = p.slot_epoch[slot];
    const uint64_t x0 = philox_w0((uint64_t)i | ((uint64_t)p.tag << 56), 0, 0, p.qid, p.k0, p.k1);
    int32_t u = (p.tag == 1)   ? (int32_t)pick_below(x0, (uint64_t)n)
                : (p.nnz > 0) ? p.col[pick_below(x0, (uint64_t)p.nnz)]
                              : p.root;
    unsigned long long *y2 = p.y2 ? p.y2 + ((i * (int64_t)p.n_blocks) / p.n_total) * n : nullptr;
    const uint64_t t0 = wall_clock64();
    int64_t len = 0;
    while (u != p.root) {
        const int32_t c = cnt[u];
        if ((uint32_t)c >= st_k(st[u], ep)) {
            raise_err(p.err, kErrInconsistent, -20);
            return;
        }
        cnt[u] = c + 1;
        const uint64_t nb = p.nbr[u];
        const uint64_t x = philox_w0((uint64_t)i, (uint64_t)u, (uint64_t)c, p.qid, p.k0, p.k1);
        if (y2) atomicAdd(&y2[u], 1ull);
        ++len;
        u = p.col[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
        if ((len & 1023) == 0 && (wall_clock64() - t0 > p.deadline || err_set(p.err))) {
            raise_err(p.err, kErrTimeout, 3);
            return;
        }
    }
    if (p.len_out) p.len_out[slot] = len;
}

hipError_t launch_loop_included(const LoopParams &p, hipStream_t s) {
    hipLaunchKernelGGL(loop_included_kernel, dim3((unsigned)((p.n_paths + 63) / 64)), dim3(64), 0, s, p);
    return hipGetLastError();
}

// Loop-included paths from node pairs (Sec. 3.4 and the resistance of Sec. 2).
// The path from s through the stacks of sample i takes, at its c-th departure
// from u, stack entry S_i[u][c]: the draw (i, u, c, qid).  Its departures from
// u, divided by d_u, estimate (L_v^{-1})_su, and
//   r(s,t) = (L_v^{-1})_ss + (L_v^{-1})_tt - 2 (L_v^{-1})_st.
// Lane l of the launch works for sample l / K (K lanes per sample) and runs
// paths q = l % K, l % K + K, ... of the 2 n_pairs paths (q even: from s_j,
// odd: from t_j, j = q / 2).  Each lane owns an n-word counter array; a word
// holds the tag of the path that last wrote it and its departure count, so a
// new path starts from zero by taking a new tag, with no clearing between
// paths.  With the Wilson trees of the launch's samples at hand, every
// departure also checks that the entry it uses was drawn by the sampler
// (c < k_u; Wilson's stacks do not depend on the start order, so the path
// from any s uses no entry the sampler did not).
__global__ __launch_bounds__(64) void pair_paths_kernel(PairParams p) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= p.n_lanes) return;
    const int64_t n = p.n;
    const int64_t slot = lane / p.lanes_per_sample;
    const int64_t i = p.sample_begin + slot;
    const uint64_t *st = p.state ? p.state + slot * n : nullptr;
    const uint32_t ep = st ? p.slot_epoch[slot] : 0u;
    uint64_t *cnt = p.cnt + lane * n;
    unsigned long long *Vb = p.V + ((i * (int64_t)p.n_blocks) / p.n_total) * p.n_pairs * 4;
    const uint64_t t0 = wall_clock64();
    unsigned long long steps = 0;
    uint32_t tag = p.tag_base;
    for (int64_t q = lane % p.lanes_per_sample; q < 2 * p.n_pairs; q += p.lanes_per_sample, ++tag) {
        const int64_t j = q >> 1;
        const bool from_t = (q & 1) != 0;
        const int32_t from = from_t ? p.pt[j] : p.ps[j];
        const int32_t other = from_t ? p.ps[j] : p.pt[j];
        int32_t u = from;
        while (u != p.root) {
            const uint64_t e = cnt[u];
            const uint32_t c = ((uint32_t)(e >> 32) == tag) ? (uint32_t)e : 0u;
            if (st ? c >= st_k(st[u], ep) : c == 0xffffffffu) {
                raise_err(p.err, kErrInconsistent, -21);
                return;
            }
            cnt[u] = ((uint64_t)tag << 32) | (uint64_t)(c + 1);
            const uint64_t nb = p.nbr[u];
            const uint64_t x = philox_w0((uint64_t)i, (uint64_t)u, (uint64_t)c, p.qid, p.k0, p.k1);
            u = p.col[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
            ++steps;
            if ((steps & 1023) == 0 && (wall_clock64() - t0 > p.deadline || err_set(p.err))) {
                raise_err(p.err, kErrTimeout, 4);
                return;
            }
        }
        // departures from the start and from the other node (the root never departs)
        const uint64_t eh = cnt[from], eo = cnt[other];
        const unsigned long long here = (from != p.root && (uint32_t)(eh >> 32) == tag) ? (uint32_t)eh : 0u;
        const unsigned long long there = (other != p.root && (uint32_t)(eo >> 32) == tag) ? (uint32_t)eo : 0u;
        unsigned long long *row = Vb + j * 4;
        if (here) atomicAdd(&row[from_t ? 2 : 0], here);
        if (there) atomicAdd(&row[from_t ? 3 : 1], there);
    }
    atomicAdd(&p.stats[kStatAbsorbed], steps);
}

hipError_t launch_pair_paths(const PairParams &p, hipStream_t s) {
    hipLaunchKernelGGL(pair_paths_kernel, dim3((unsigned)((p.n_lanes + 63) / 64)), dim3(64), 0, s, p);
    return hipGetLastError();
}

// Number of i in [0, omega) with floor(i * B / omega) == b.
__device__ __forceinline__ int64_t pair_block_count(int64_t omega, int32_t B, int32_t b) {
    const int64_t lo = ((int64_t)b * omega + B - 1) / B;
    const int64_t hi = ((int64_t)(b + 1) * omega + B - 1) / B;
    return hi - lo;
}

// FP64 assembly, one lane per pair, from the exact sums V:
//   (L_v^{-1})_ss = V0 / (omega d_s),  (L_v^{-1})_tt = V2 / (omega d_t),
//   (L_v^{-1})_st = (V1 / d_t + V3 / d_s) / (2 omega)   (both orders of the symmetric entry),
//   r(s,t) = (V0 / d_s - V1 / d_t + V2 / d_t - V3 / d_s) / omega,
// and the batch-means standard error of r over the B sample blocks.
__global__ __launch_bounds__(64) void pair_assemble_kernel(PairAsmParams p) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= p.n_pairs) return;
    const double ds = (double)nbr_deg(p.nbr[p.ps[j]]);
    const double dt = (double)nbr_deg(p.nbr[p.pt[j]]);
    unsigned long long a[4] = {0, 0, 0, 0};
    double m = 0.0, m2 = 0.0;
    for (int b = 0; b < p.B; ++b) {
        const unsigned long long *vb = p.V + ((int64_t)b * p.n_pairs + j) * 4;
        for (int k = 0; k < 4; ++k) a[k] += vb[k];
        if (p.B > 1) {
            const double nb = (double)pair_block_count(p.omega, p.B, b);
            const double rb = ((double)vb[0] / ds - (double)vb[1] / dt + (double)vb[2] / dt - (double)vb[3] / ds) / nb;
            const double d = rb - m;
            m += d / (b + 1);
            m2 += d * (rb - m);
        }
    }
    const double om = (double)p.omega;
    if (p.r) p.r[j] = ((double)a[0] / ds - (double)a[1] / dt + (double)a[2] / dt - (double)a[3] / ds) / om;
    if (p.r_se) p.r_se[j] = (p.B > 1) ? sqrt(m2 / (p.B - 1)) / sqrt((double)p.B) : __builtin_nan("");
    if (p.lv) {
        p.lv[3 * j + 0] = (double)a[0] / (om * ds);
        p.lv[3 * j + 1] = ((double)a[1] / dt + (double)a[3] / ds) / (2.0 * om);
        p.lv[3 * j + 2] = (double)a[2] / (om * dt);
    }
}

hipError_t launch_pair_assemble(const PairAsmParams &p, hipStream_t s) {
    if (p.n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_assemble_kernel, dim3((unsigned)((p.n_pairs + 63) / 64)), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
