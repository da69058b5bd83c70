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
    if (p.stats) atomicAdd(&p.stats[kStatAbsorbed], (unsigned long long)len);
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
// Work item slot * 2 n_pairs + q: path q (q even: from s_j, odd: from t_j,
// j = q / 2) through the stacks of sample sample_begin + slot.  In the rows
// form there is one path per source (item slot * n_pairs + j, from s_j), and
// every departure from u adds one to the source's row at u instead.
//
// Path lengths spread widely, so a lane does not wait for the other lanes of
// its wave: whenever its path ends it takes the next item, from one of
// n_parts counters (workgroup b uses part b mod n_parts), one atomic per wave
// for all lanes that need an item.
//
// A lane keeps the departure counts of its current path in one of two forms:
//   dense  one 8-byte word per node (tag << 32 | count);
//   hashed an open-addressing table of 2^hash_log2 words (node | tag << 32 |
//          count << 48), probed linearly from a multiplicative hash; a path
//          that meets more than hash_limit distinct nodes, or departs 2^16-1
//          times from one node, is abandoned and queued for the dense form
//          (in the rows form, after its departures so far are taken back out
//          of its row; the table holds exactly those).
// A word belongs to the current path only if it carries the path's tag, so a
// new path starts from zero by taking the lane's next tag; only when the tags
// run out does a lane clear its own words.  Each lane's last tag persists in
// lane_tag between launches.  With the Wilson trees of the launch's samples
// at hand, every departure also checks that the entry it uses was drawn by the
// sampler (c < k_u: Wilson's stacks do not depend on the start order, so the
// path from any s uses no entry the sampler did not).
constexpr uint32_t kDepFull = 0xffffffffu;

struct DenseDepartures {
    uint64_t *w;
    int64_t words;
    uint32_t tag;
    static constexpr uint32_t kTagMax = 0xffffffffu;
    __device__ __forceinline__ void clear() {
        for (int64_t k = 0; k < words; ++k) w[k] = 0ull;
    }
    __device__ __forceinline__ void start(uint32_t t) { tag = t; }
    __device__ __forceinline__ uint32_t get(int32_t u) const {
        const uint64_t e = w[u];
        return ((uint32_t)(e >> 32) == tag) ? (uint32_t)e : 0u;
    }
    // take the current path's departures back out of a row
    __device__ void unwind(unsigned long long *row) const {
        for (int64_t k = 0; k < words; ++k) {
            const uint64_t e = w[k];
            if ((uint32_t)(e >> 32) == tag && (uint32_t)e) atomicAdd(&row[k], 0ull - (unsigned long long)(uint32_t)e);
        }
    }
    // count before this departure from u, or kDepFull
    __device__ __forceinline__ uint32_t bump(int32_t u) {
        const uint32_t c = get(u);
        if (c == kDepFull - 1) return kDepFull;
        w[u] = ((uint64_t)tag << 32) | (uint64_t)(c + 1);
        return c;
    }
};

struct HashDepartures {
    uint64_t *w;
    int64_t words;
    uint32_t mask, shift, tag;
    int32_t distinct, limit;
    static constexpr uint32_t kTagMax = 0xffffu;
    __device__ __forceinline__ void clear() {
        for (int64_t k = 0; k < words; ++k) w[k] = 0ull;
    }
    __device__ __forceinline__ void start(uint32_t t) {
        tag = t;
        distinct = 0;
    }
    __device__ __forceinline__ uint32_t home(int32_t u) const { return ((uint32_t)u * 2654435761u) >> shift; }
    __device__ __forceinline__ bool mine(uint64_t e) const { return (uint32_t)((e >> 32) & 0xffffu) == tag; }
    __device__ __forceinline__ uint32_t get(int32_t u) const {
        for (uint32_t h = home(u);; h = (h + 1) & mask) {   // ends: at most `limit` < 2^hash_log2 words are the path's
            const uint64_t e = w[h];
            if (!mine(e)) return 0u;
            if ((uint32_t)e == (uint32_t)u) return (uint32_t)(e >> 48);
        }
    }
    // take the current path's departures back out of a row
    __device__ void unwind(unsigned long long *row) const {
        for (int64_t k = 0; k < words; ++k) {
            const uint64_t e = w[k];
            if (mine(e)) atomicAdd(&row[(uint32_t)e], 0ull - (unsigned long long)(e >> 48));
        }
    }
    __device__ __forceinline__ uint32_t bump(int32_t u) {
        for (uint32_t h = home(u);; h = (h + 1) & mask) {
            const uint64_t e = w[h];
            if (!mine(e)) {
                if (++distinct > limit) return kDepFull;
                w[h] = (uint64_t)(uint32_t)u | ((uint64_t)tag << 32) | (1ull << 48);
                return 0u;
            }
            if ((uint32_t)e == (uint32_t)u) {
                const uint32_t c = (uint32_t)(e >> 48);
                if (c == 0xffffu) return kDepFull;
                w[h] = (e & 0x0000ffffffffffffull) | ((uint64_t)(c + 1) << 48);
                return c;
            }
        }
    }
};

template <class Dep>
__device__ void pair_lane(const PairParams &p, Dep &dep, int64_t lane) {
    const int64_t n = p.n;
    const int64_t paths = p.rows ? p.n_pairs : 2 * p.n_pairs;
    const int part = (int)(blockIdx.x % (unsigned)p.n_parts);
    const int64_t n_items = p.queue_in ? (int64_t)*p.queue_in_len : p.n_items;
    const int64_t lo = n_items * part / p.n_parts, hi = n_items * (part + 1) / p.n_parts;
    unsigned long long *next = p.next + 16 * part;   // one 128-byte line per part
    const uint64_t t0 = wall_clock64();
    const int wl = (int)(threadIdx.x & 63);
    unsigned long long steps = 0;
    uint32_t tag = p.lane_tag[lane];
    // current path
    int64_t item = -1, j = 0, i = 0;
    int32_t u = p.root, from = 0, other = 0;
    bool from_t = false;
    const uint64_t *st = nullptr;
    uint32_t ep = 0;
    unsigned long long *row = nullptr;   // rows form: the current path's row
    for (;;) {
        if (u == p.root && item >= 0 && p.rows) {
            item = -1;   // rows form: the departures went to the row as they happened
        } else if (u == p.root && item >= 0) {
            // the path reached v: add its departures from s_j and t_j (the root never departs)
            const unsigned long long here = (from != p.root) ? dep.get(from) : 0u;
            const unsigned long long there = (other != p.root) ? dep.get(other) : 0u;
            unsigned long long *vrow = p.V + (((i * (int64_t)p.n_blocks) / p.n_total) * p.n_pairs + j) * 4;
            if (here) atomicAdd(&vrow[from_t ? 2 : 0], here);
            if (there) atomicAdd(&vrow[from_t ? 3 : 1], there);
            item = -1;
        }
        const bool need = (u == p.root);
        const unsigned long long want = __ballot(need);
        if (want) {
            const int leader = __ffsll((long long)want) - 1;
            unsigned long long base = 0;
            if (wl == leader) base = atomicAdd(next, (unsigned long long)__popcll(want));
            base = __shfl(base, leader);
            if (need) {
                const int64_t e = lo + (int64_t)base + __popcll(want & ((1ull << wl) - 1ull));
                if (e >= hi) break;
                item = p.queue_in ? (int64_t)p.queue_in[e] : e;
                const int64_t slot = item / paths, q = item % paths;
                i = p.sample_begin + slot;
                st = p.state ? p.state + slot * n : nullptr;
                ep = st ? p.slot_epoch[slot] : 0u;
                if (p.rows) {
                    j = q;
                    from_t = false;
                    from = other = p.ps[j];
                    row = p.rows + (((i * (int64_t)p.n_blocks) / p.n_total) * p.n_pairs + j) * n;
                } else {
                    j = q >> 1;
                    from_t = (q & 1) != 0;
                    from = from_t ? p.pt[j] : p.ps[j];
                    other = from_t ? p.ps[j] : p.pt[j];
                }
                if (tag == Dep::kTagMax) {   // tags used up: clear this lane's words
                    dep.clear();
                    tag = 0;
                }
                dep.start(++tag);
                u = from;
                continue;   // a path from the root ends at once
            }
        }
        // one departure from u
        const uint64_t nb = p.nbr[u];   // independent of the count: in flight with the probe
        const uint64_t sw = st ? st[u] : 0ull;
        const uint32_t c = dep.bump(u);
        if (c == kDepFull) {
            if (!p.queue_out) {   // dense form: 2^32-1 departures from one node
                raise_err(p.err, kErrDrawOverflow, -22);
                break;
            }
            // rows form: the departures so far already went to the row
            if (row) dep.unwind(row);
            const unsigned long long at = atomicAdd(p.queue_out_len, 1ull);
            p.queue_out[at] = (unsigned long long)item;   // capacity: every item of the launch
            item = -1;
            u = p.root;
            continue;
        }
        if (st && c >= st_k(sw, ep)) {
            raise_err(p.err, kErrInconsistent, -21);
            break;
        }
        if (row) atomicAdd(&row[u], 1ull);
        const uint64_t x = philox_w0((uint64_t)i, (uint64_t)u, (uint64_t)c, p.qid, p.k0, p.k1);
        u = p.col[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
        ++steps;
        if ((steps & 1023) == 0 && (wall_clock64() - t0 > p.deadline || err_set(p.err))) {
            raise_err(p.err, kErrTimeout, 4);
            break;
        }
    }
    p.lane_tag[lane] = tag;
    atomicAdd(&p.stats[kStatAbsorbed], steps);
}

__global__ __launch_bounds__(64) void pair_paths_hash_kernel(PairParams p) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= p.n_lanes) return;
    HashDepartures dep;
    dep.words = (int64_t)1 << p.hash_log2;
    dep.w = p.tbl + lane * dep.words;
    dep.mask = (1u << p.hash_log2) - 1u;
    dep.shift = 32u - (uint32_t)p.hash_log2;
    dep.limit = p.hash_limit;
    dep.tag = 0;
    dep.distinct = 0;
    pair_lane(p, dep, lane);
}

__global__ __launch_bounds__(64) void pair_paths_dense_kernel(PairParams p) {
    const int64_t lane = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (lane >= p.n_lanes) return;
    DenseDepartures dep;
    dep.words = p.n;
    dep.w = p.cnt + lane * p.n;
    dep.tag = 0;
    pair_lane(p, dep, lane);
}

hipError_t launch_pair_paths(const PairParams &p, bool hashed, hipStream_t s) {
    if (p.n_lanes <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((p.n_lanes + 63) / 64);
    if (hashed)
        hipLaunchKernelGGL(pair_paths_hash_kernel, dim3(blocks), dim3(64), 0, s, p);
    else
        hipLaunchKernelGGL(pair_paths_dense_kernel, dim3(blocks), dim3(64), 0, s, p);
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

// Whole rows: (L_v^{-1})_{s_j u} = sum over blocks of the departures from u
// on the paths from s_j, over (omega d_u); column v stays zero.
__global__ __launch_bounds__(256) void lv_rows_kernel(const unsigned long long *Y, const uint64_t *nbr, int64_t n,
                                                      int64_t n_src, int32_t B, int64_t omega, int32_t root,
                                                      double *out) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n_src * n; e += stride) {
        const int64_t u = e % n;
        unsigned long long a = 0;
        for (int b = 0; b < B; ++b) a += Y[(int64_t)b * n_src * n + e];
        out[e] = (u == root) ? 0.0 : (double)a / ((double)omega * (double)nbr_deg(nbr[u]));
    }
}

hipError_t launch_lv_rows(const unsigned long long *Y, const uint64_t *nbr, int64_t n, int64_t n_src, int32_t B,
                          int64_t omega, int32_t root, double *out, hipStream_t s) {
    const int64_t total = n_src * n;
    if (total <= 0) return hipSuccess;
    int64_t grid = (total + 255) / 256;
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(lv_rows_kernel, dim3((unsigned)grid), dim3(256), 0, s, Y, nbr, n, n_src, B, omega, root, out);
    return hipGetLastError();
}

hipError_t launch_pair_assemble(const PairAsmParams &p, hipStream_t s) {
    if (p.n_pairs <= 0) return hipSuccess;
    hipLaunchKernelGGL(pair_assemble_kernel, dim3((unsigned)((p.n_pairs + 63) / 64)), dim3(64), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
