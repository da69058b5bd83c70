// Wilson loop-erased-walk sampling rooted at the landmark v (Sec. 3.4; the
// sampling phase of Alg. 2 and the y1 walk of Alg. 4), in four execution forms:
//
//  wilson_lane_kernel  one lane per sample; walks started from the nodes in
//                      ascending order, each walk followed until it meets
//                      the tree and then retraced (the paper's sequential
//                      loop).  Simple, latency bound; kept as a reference
//                      schedule and for tiny graphs.
//
//  wilson_wave_kernel  one wavefront per sample with 64 walkers in lockstep.
//                      Draws are keyed to per-node stack entries, so by
//                      Wilson's stack argument any order of popping cycles
//                      gives the same stacks, draw counts and tree.  The
//                      walkers therefore run concurrently:
//                        - a walker claims the nodes on its current path
//                          (tag = lane+1); arriving at its own path closes a
//                          loop, which it releases (those entries are popped)
//                          before drawing again at the loop's entry;
//                        - arriving at a node on another walker's path parks
//                          the walker until that node is released or joins
//                          the tree;
//                        - parked walkers that wait on each other in a ring
//                          form one cycle of stack tops across several paths;
//                          it is found by pointer jumping over the 64 lanes
//                          and popped as a unit: each walker resumes at the
//                          node where the previous walker of the ring waits;
//                        - reaching the tree retraces the path and marks it.
//                      Idle walkers take new starts from a coalesced scan of
//                      the node range and from a small LDS list of released
//                      nodes the scan has already passed.
//
//  wilson_group_kernel the wave form's protocol over W = 2, 4 or 8 wavefronts
//                      of one workgroup (64 W walkers per sample), for runs
//                      with too few samples to fill the device.
//
//  wilson_lds_kernel   the lane form with the CSR and the lanes' state in
//                      LDS, for graphs of at most 1024 nodes.
//
// The lane, wave and workgroup forms keep one packed 64-bit word per node per
// sample slot in HBM (next, draw count, tag, epoch); every form records each
// sample's total draws.  Every node
// other than v draws at least once per sample, so when a node joins the tree
// only its draws beyond the first, k - 1, are added to the per-block count
// array; the one-per-sample baseline is added back when counts are read out
// (lap_sample_forests) or assembled.
#include <algorithm>

#include "lap_device.h"
#include "lap_launch.h"
#include "group_sample.h"
#include "wave_sample.h"

namespace lap {

__device__ __forceinline__ void keep_slot_init(const WilsonParams &p, int keep_q) {
    if (keep_q < 0) return;
    if (p.next_out) p.next_out[(int64_t)keep_q * p.n + p.root] = -1;
    if (p.draws_out) p.draws_out[(int64_t)keep_q * p.n + p.root] = 0;
}

__device__ __forceinline__ int find_keep(const WilsonParams &p, int64_t sample) {
    int q = -1;
    for (int i = 0; i < p.n_keep; ++i)
        if (p.keep_idx[i] == sample) q = i;
    return q;
}

// ----------------------------------------------------------------- lane form
__global__ __launch_bounds__(64) void wilson_lane_kernel(WilsonParams p) {
    const int64_t slot = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t slots = p.n_slots;
    if (slot >= p.n_slots || slot >= p.n_samples) return;
    const int64_t n = p.n;
    uint64_t *st = p.state + slot * n;
    uint32_t ep = p.slot_epoch[slot];
    const uint64_t t0 = wall_clock64();
    unsigned long long draws_all = 0, trees = 0;
    bool stop = false;
    for (int64_t smp = slot; smp < p.n_samples && !stop; smp += slots) {
        const int64_t sample = p.sample_begin + smp;
        ep ^= 1u;
        const int keep_q = find_keep(p, sample);
        unsigned long long *y1b = p.y1 ? p.y1 + block_of(sample, p.n_blocks, p.n_total) * n : nullptr;
        st[p.root] = st_pack(-1, 0, kTagTree, ep);
        keep_slot_init(p, keep_q);
        int64_t y1 = 0;
        uint64_t it = 0;
        for (int64_t u = 0; u < n && !stop; ++u) {
            if (u == p.root) continue;
            uint64_t wu = st[u];
            if (st_tag(wu, ep) == kTagTree) continue;
            // walk from u until the tree is hit; next[] is overwritten, so
            // loops erase themselves
            int32_t cur = (int32_t)u;
            uint32_t kc = st_k(wu, ep);
            uint64_t nb = p.nbr[cur];
            while (true) {
                const uint64_t x = philox_w0((uint64_t)sample, (uint64_t)cur, kc, p.qid, p.k0, p.k1);
                const int32_t w = p.col[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
                if (kc >= kMaxDraws) { raise_err(p.err, kErrDrawOverflow, cur); stop = true; break; }
                st[cur] = st_pack(w, kc + 1, 1, ep);
                ++y1;
                const uint64_t ww = st[w];
                if (st_tag(ww, ep) == kTagTree) break;
                cur = w;
                kc = st_k(ww, ep);
                nb = p.nbr[w];
                if ((++it & 1023) == 0 && (wall_clock64() - t0 > p.deadline || err_set(p.err))) {
                    raise_err(p.err, kErrTimeout, 0);
                    stop = true;
                    break;
                }
            }
            if (stop) break;
            // retrace from u: the loop-erased path joins the tree
            int32_t y = (int32_t)u;
            while (true) {
                const uint64_t wy = st[y];
                if (st_tag(wy, ep) == kTagTree) break;
                const uint32_t k = st_k(wy, ep);
                const int32_t nx = st_next(wy);
                st[y] = st_pack(nx, k, kTagTree, ep);
                if (y1b && k > 1) atomicAdd(&y1b[y], (unsigned long long)(k - 1));
                if (keep_q >= 0) {
                    if (p.next_out) p.next_out[(int64_t)keep_q * n + y] = nx;
                    if (p.draws_out) p.draws_out[(int64_t)keep_q * n + y] = (int32_t)k;
                }
                y = nx;
            }
        }
        if (stop) break;
        if (p.y1_per_sample) p.y1_per_sample[smp] = y1;
        draws_all += (unsigned long long)y1;
        ++trees;
    }
    p.slot_epoch[slot] = ep;
    atomicAdd(&p.stats[kStatDraws], draws_all);
    atomicAdd(&p.stats[kStatTrees], trees);
}

// ------------------------------------------------------------- LDS lane form
// One lane per sample, as the lane form, for graphs small enough that the CSR
// and one 32-bit state word per node for every lane of the workgroup fit in
// LDS (layout and word format beside kLdsMaxNodes).  A lane is in one of three
// phases: scanning for the next start node, walking (one draw per round, the
// only step that evaluates the generator) or retracing a finished walk into
// the tree.  Scans and retraces advance in an inner loop until the lane needs
// a draw, so the rounds a wavefront spends on Philox are the draws of its
// longest sample rather than its longest sample's draws, scan and retrace
// steps together.  Each lane clears its own state column at the start of a
// sample, so no epoch is kept; lanes loop over samples with the grid's stride.
__global__ __launch_bounds__(64) void wilson_lds_kernel(WilsonParams p) {
    extern __shared__ uint32_t lds[];
    const int S = (int)blockDim.x;
    const int lane = (int)threadIdx.x;
    const int32_t n = (int32_t)p.n;
    uint32_t *rp = lds;
    uint16_t *col = reinterpret_cast<uint16_t *>(lds + n + 1);
    uint32_t *st = lds + lds_state_offset(p.n, p.nnz);
    for (int32_t u = lane; u < n; u += S) rp[u] = (uint32_t)nbr_off(p.nbr[u]);
    if (lane == 0) rp[n] = (uint32_t)p.nnz;
    for (int64_t j = lane; j < p.nnz; j += S) col[j] = (uint16_t)p.col[j];
    __syncthreads();

    enum : int { kScan = 0, kWalk = 1, kRetrace = 2, kDone = 3 };
    const uint64_t t0 = wall_clock64();
    const int64_t stride = (int64_t)gridDim.x * S;
    int64_t smp = (int64_t)blockIdx.x * S + lane;
    int64_t sample = 0, y1 = 0;
    int keep_q = -1;
    unsigned long long *y1b = nullptr;
    int mode = kDone;
    int32_t u = 0, cur = 0, start = 0, y = 0, rsteps = 0;
    uint32_t kc = 0;
    unsigned long long draws_all = 0, trees = 0;

    auto begin_sample = [&]() {
        if (smp >= p.n_samples) {
            mode = kDone;
            return;
        }
        sample = p.sample_begin + smp;
        keep_q = find_keep(p, sample);
        y1b = p.y1 ? p.y1 + block_of(sample, p.n_blocks, p.n_total) * p.n : nullptr;
        for (int32_t v = 0; v < n; ++v) st[v * S + lane] = 0u;
        st[p.root * S + lane] = kLdsTree;
        keep_slot_init(p, keep_q);
        y1 = 0;
        u = 0;
        mode = kScan;
    };
    begin_sample();

    uint64_t it = 0;
    while (true) {
        // scans and retraces until this lane needs a draw
        while (mode == kScan || mode == kRetrace) {
            if (mode == kScan) {
                if (u >= n) {
                    if (p.y1_per_sample) p.y1_per_sample[smp] = y1;
                    draws_all += (unsigned long long)y1;
                    ++trees;
                    smp += stride;
                    begin_sample();
                    continue;
                }
                const uint32_t w = st[u * S + lane];
                if (w & kLdsTree) {
                    ++u;
                    continue;
                }
                cur = start = u;
                kc = w >> kLdsKShift;
                mode = kWalk;
            } else {
                const uint32_t w = st[y * S + lane];
                if (w & kLdsTree) {
                    mode = kScan;
                    continue;
                }
                if (++rsteps > n) {   // a path has at most n - 1 nodes off the tree
                    raise_err(p.err, kErrInconsistent, -1);
                    mode = kDone;
                    break;
                }
                const uint32_t k = w >> kLdsKShift;
                const int32_t nx = (int32_t)(w & (kLdsTree - 1u));
                st[y * S + lane] = w | kLdsTree;
                if (y1b && k > 1) atomicAdd(&y1b[y], (unsigned long long)(k - 1));
                if (keep_q >= 0) {
                    if (p.next_out) p.next_out[(int64_t)keep_q * n + y] = nx;
                    if (p.draws_out) p.draws_out[(int64_t)keep_q * n + y] = (int32_t)k;
                }
                y = nx;
            }
        }
        if (!__any(mode == kWalk)) break;
        if (mode == kWalk) {
            if (kc >= kMaxDraws) {
                raise_err(p.err, kErrDrawOverflow, cur);
                mode = kDone;
            } else {
                const uint64_t x = philox_w0((uint64_t)sample, (uint64_t)cur, kc, p.qid, p.k0, p.k1);
                const uint32_t r0 = rp[cur];
                const int32_t w = (int32_t)col[r0 + (uint32_t)pick_below(x, (uint64_t)(rp[cur + 1] - r0))];
                st[cur * S + lane] = (uint32_t)w | ((kc + 1) << kLdsKShift);
                ++y1;
                const uint32_t sw = st[w * S + lane];
                if (sw & kLdsTree) {
                    mode = kRetrace;
                    y = start;
                    rsteps = 0;
                } else {
                    cur = w;
                    kc = sw >> kLdsKShift;
                }
            }
        }
        // the time limit and other lanes' errors, checked by every lane alike
        if ((++it & 1023) == 0 && (wall_clock64() - t0 > p.deadline || err_set(p.err))) {
            raise_err(p.err, kErrTimeout, 0);
            break;
        }
    }
    atomicAdd(&p.stats[kStatDraws], draws_all);
    atomicAdd(&p.stats[kStatTrees], trees);
}

// ----------------------------------------------------------------- wave form
// ARCS: draws read the arc record {target, target's adjacency record} of the
// drawn column slot, so an arrival loads only the target's state word.
template <bool ARCS>
__global__ __launch_bounds__(64) void wilson_wave_kernel(WilsonParams p) {
    __shared__ WaveShared sh;
    const int lane = (int)threadIdx.x;
    const int64_t slot = blockIdx.x;
    WaveSampleArgs c;
    c.n = p.n;
    c.nnz = p.nnz;
    c.nbr = p.nbr;
    c.col = p.col;
    c.arcs = p.arcs;
    c.root = p.root;
    c.k0 = p.k0;
    c.k1 = p.k1;
    c.qid = p.qid;
    c.st = p.state + slot * p.n;
    c.err = p.err;
    c.t0 = wall_clock64();
    c.deadline = p.deadline;
    c.scan_offset = p.scan_offset;
    uint32_t ep = p.slot_epoch[slot];
    WaveStats ws;
    for (int64_t smp = slot; smp < p.n_samples; smp += gridDim.x) {
        const int64_t sample = p.sample_begin + smp;
        ep ^= 1u;
        const int keep_q = find_keep(p, sample);
        c.sample = sample;
        c.ep = ep;
        c.y1b = p.y1 ? p.y1 + block_of(sample, p.n_blocks, p.n_total) * p.n : nullptr;
        c.keep_next = (keep_q >= 0 && p.next_out) ? p.next_out + (int64_t)keep_q * p.n : nullptr;
        c.keep_draws = (keep_q >= 0 && p.draws_out) ? p.draws_out + (int64_t)keep_q * p.n : nullptr;
        int64_t y1 = 0;
        if (!wave_wilson_sample<ARCS>(c, sh, &y1, ws)) break;
        if (lane == 0) {
            if (p.y1_per_sample) p.y1_per_sample[smp] = y1;
            ++ws.trees;
        }
    }
    if (lane == 0) p.slot_epoch[slot] = ep;
    flush_wave_stats(ws, p.stats);
}

// ------------------------------------------------------------ workgroup form
// W wavefronts per sample (group_sample.h); one workgroup per slot.
// (at least 4 waves per SIMD: 16 per CU, as in the wave form)
template <int W, bool ARCS>
__global__ __launch_bounds__(kWave * W, 4) void wilson_group_kernel(WilsonParams p) {
    __shared__ GroupShared<W> sh;
    const int tid = (int)threadIdx.x;
    const int64_t slot = blockIdx.x;
    WaveSampleArgs c;
    c.n = p.n;
    c.nnz = p.nnz;
    c.nbr = p.nbr;
    c.col = p.col;
    c.arcs = p.arcs;
    c.root = p.root;
    c.k0 = p.k0;
    c.k1 = p.k1;
    c.qid = p.qid;
    c.st = p.state + slot * p.n;
    c.err = p.err;
    c.t0 = wall_clock64();
    c.deadline = p.deadline;
    c.scan_offset = p.scan_offset;
    uint32_t ep = p.slot_epoch[slot];
    WaveStats ws;
    for (int64_t smp = slot; smp < p.n_samples; smp += gridDim.x) {
        const int64_t sample = p.sample_begin + smp;
        ep ^= 1u;
        const int keep_q = find_keep(p, sample);
        c.sample = sample;
        c.ep = ep;
        c.y1b = p.y1 ? p.y1 + block_of(sample, p.n_blocks, p.n_total) * p.n : nullptr;
        c.keep_next = (keep_q >= 0 && p.next_out) ? p.next_out + (int64_t)keep_q * p.n : nullptr;
        c.keep_draws = (keep_q >= 0 && p.draws_out) ? p.draws_out + (int64_t)keep_q * p.n : nullptr;
        int64_t y1 = 0;
        if (!group_wilson_sample<W, ARCS>(c, sh, &y1, ws)) break;
        if (tid == 0) {
            if (p.y1_per_sample) p.y1_per_sample[smp] = y1;
            ++ws.trees;
        }
    }
    if (tid == 0) p.slot_epoch[slot] = ep;
    flush_group_stats(ws, p.stats);
}

// ----------------------------------------------------------------- launchers
hipError_t launch_wilson_lane(const WilsonParams &p, int64_t slots, hipStream_t s) {
    const int bs = 64;
    const int64_t grid = (slots + bs - 1) / bs;
    hipLaunchKernelGGL(wilson_lane_kernel, dim3((unsigned)grid), dim3(bs), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wilson_lds(const WilsonParams &p, int lanes, int64_t slots, hipStream_t s) {
    if (lanes < 1 || lanes > 64 || p.n > kLdsMaxNodes) return hipErrorInvalidValue;
    const int64_t need = (std::min(slots, p.n_samples) + lanes - 1) / lanes;
    const unsigned grid = (unsigned)std::min<int64_t>(std::max<int64_t>(need, 1), (int64_t)1 << 16);
    const size_t bytes = (size_t)lds_bytes(p.n, p.nnz, lanes);
    hipError_t e = hipFuncSetAttribute((const void *)wilson_lds_kernel, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bytes);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(wilson_lds_kernel, dim3(grid), dim3(lanes), bytes, s, p);
    return hipGetLastError();
}

hipError_t launch_wilson_wave(const WilsonParams &p, int64_t slots, hipStream_t s) {
    if (p.arcs)
        hipLaunchKernelGGL(wilson_wave_kernel<true>, dim3((unsigned)slots), dim3(kWave), 0, s, p);
    else
        hipLaunchKernelGGL(wilson_wave_kernel<false>, dim3((unsigned)slots), dim3(kWave), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap

namespace lap {

template <bool ARCS>
static hipError_t launch_group_form(const WilsonParams &p, int64_t slots, int waves, hipStream_t s) {
    switch (waves) {
    case 2:
        hipLaunchKernelGGL((wilson_group_kernel<2, ARCS>), dim3((unsigned)slots), dim3(kWave * 2), 0, s, p);
        break;
    case 4:
        hipLaunchKernelGGL((wilson_group_kernel<4, ARCS>), dim3((unsigned)slots), dim3(kWave * 4), 0, s, p);
        break;
    case 8:
        hipLaunchKernelGGL((wilson_group_kernel<8, ARCS>), dim3((unsigned)slots), dim3(kWave * 8), 0, s, p);
        break;
    default:
        return hipErrorInvalidValue;
    }
    return hipGetLastError();
}

hipError_t launch_wilson_group(const WilsonParams &p, int64_t slots, int waves, hipStream_t s) {
    return p.arcs ? launch_group_form<true>(p, slots, waves, s) : launch_group_form<false>(p, slots, waves, s);
}

}  // namespace lap
