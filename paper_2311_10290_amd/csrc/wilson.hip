// Wilson loop-erased-walk sampling rooted at the landmark v (Sec. 3.4; the
// sampling phase of Alg. 2 and the y1 walk of Alg. 4), two execution forms:
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
// Both keep one packed 64-bit word per node per sample slot in HBM (next,
// draw count, tag, epoch), add each node's final draw count into the
// per-block count array when the node joins the tree, and record each
// sample's total draws.
#include "lap_device.h"
#include "lap_launch.h"

namespace lap {

constexpr int kWave = 64;
constexpr int kClaimBits = 11;
constexpr int kClaimMask = (1 << kClaimBits) - 1;
constexpr int kRevCap = 256;

enum : int32_t { kIdle = 0, kDraw = 1, kArrive = 2, kRetrace = 3, kRelease = 4, kPopLoad = 5 };

__device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int64_t block_of(int64_t sample, int32_t B, int64_t n_total) {
    return (sample * (int64_t)B) / n_total;
}

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
                if (y1b) atomicAdd(&y1b[y], (unsigned long long)k);
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

// ----------------------------------------------------------------- wave form
__global__ __launch_bounds__(64) void wilson_wave_kernel(WilsonParams p) {
    __shared__ uint8_t claim_tbl[1 << kClaimBits];
    __shared__ int32_t rev[kRevCap];
    __shared__ int32_t cand[2 * kWave];
    __shared__ int32_t ent[kWave];
    __shared__ int32_t mark[kWave];
    __shared__ int64_t cut_at;

    const int lane = (int)threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t n = p.n;
    const int64_t slot = blockIdx.x;
    uint64_t *st = p.state + slot * n;
    uint32_t ep = p.slot_epoch[slot];
    const uint64_t t0 = wall_clock64();
    unsigned long long s_iters = 0, s_draws = 0, s_trees = 0, s_pops = 0, s_rescans = 0;
    bool stop = false;

    for (int64_t smp = slot; smp < p.n_samples && !stop; smp += gridDim.x) {
        const int64_t sample = p.sample_begin + smp;
        ep ^= 1u;
        const int keep_q = find_keep(p, sample);
        unsigned long long *y1b = p.y1 ? p.y1 + block_of(sample, p.n_blocks, p.n_total) * n : nullptr;
        if (lane == 0) {
            st[p.root] = st_pack(-1, 0, kTagTree, ep);
            keep_slot_init(p, keep_q);
        }
        __syncthreads();

        int64_t cursor = 0;        // next node id the scan looks at (wave-uniform)
        int rev_n = 0;             // entries in rev[] (wave-uniform)
        bool overflow = false;     // rev[] overflowed: rescan needed (wave-uniform)
        int64_t tree_local = (lane == 0) ? 1 : 0;
        int64_t y1_local = 0;
        int mode = kIdle;
        bool is_start = false;     // the ARRIVE target is a start candidate
        bool fresh = false;        // mode was set by this iteration's scan
        int32_t s = -1, h = -1, w = -1, x = -1, stop_at = -1, e = -1;
        uint32_t kh = 0, ke = 0;
        uint64_t nbh = 0, nbe = 0;
        uint64_t it = 0;

        while (true) {
            ++it;
            if ((it & 255) == 0) {
                int bad = (wall_clock64() - t0 > p.deadline) ? 2 : (err_set(p.err) ? 1 : 0);
                bad = __builtin_amdgcn_readfirstlane(bad);
                if (bad) {
                    if (bad == 2) raise_err(p.err, kErrTimeout, 0);
                    stop = true;
                    break;
                }
            }
            // ---- 1. idle walkers take released nodes the scan has passed
            const uint64_t idle = __ballot(mode == kIdle);
            const int n_idle = __popcll(idle);
            bool scanning = false;
            if (n_idle > 0) {
                const int take = min(n_idle, rev_n);
                if (mode == kIdle) {
                    const int r = __popcll(idle & below);
                    if (r < take) {
                        w = rev[rev_n - 1 - r];
                        mode = kArrive;
                        is_start = true;
                    }
                }
                rev_n -= take;
                scanning = (n_idle > take) && (cursor < n);
            }

            // ---- 2. one round of loads for every walker (+ the scan)
            int64_t ld_st = -1, ld_nb = -1, ld_col = -1;
            if (mode == kDraw) {
                const uint64_t r = philox_w0((uint64_t)sample, (uint64_t)h, kh, p.qid, p.k0, p.k1);
                ld_col = nbr_off(nbh) + (int64_t)pick_below(r, nbr_deg(nbh));
            } else if (mode == kArrive) {
                ld_st = w;
                ld_nb = w;
            } else if (mode == kRetrace || mode == kRelease) {
                ld_st = x;
            } else if (mode == kPopLoad) {
                ld_st = e;
                ld_nb = e;
            }
            // every index must stay inside the graph; anything else is a bug and
            // stops the kernel instead of touching memory out of bounds
            const bool need_st = mode == kArrive || mode == kRetrace || mode == kRelease || mode == kPopLoad;
            const bool oob = (need_st && (ld_st < 0 || ld_st >= n)) || (ld_nb >= n) ||
                             (mode == kDraw && (h < 0 || h >= n || ld_col < 0 || ld_col >= p.nnz));
            if (__ballot(oob)) {
                if (oob) raise_err(p.err, kErrInconsistent, -1);
                stop = true;
                break;
            }
            const int64_t sc0 = cursor + lane, sc1 = cursor + kWave + lane;
            const uint64_t v_st = (ld_st >= 0) ? st[ld_st] : 0ull;
            const uint64_t v_nb = (ld_nb >= 0) ? p.nbr[ld_nb] : 0ull;
            const int32_t v_col = (ld_col >= 0) ? p.col[ld_col] : 0;
            const uint64_t v_s0 = (scanning && sc0 < n) ? st[sc0] : 0ull;
            const uint64_t v_s1 = (scanning && sc1 < n) ? st[sc1] : 0ull;

            // ---- 3. scan: hand FREE candidates to the remaining idle walkers
            if (scanning) {
                const bool f0 = sc0 < n && st_tag(v_s0, ep) == kTagFree;
                const bool f1 = sc1 < n && st_tag(v_s1, ep) == kTagFree;
                const uint64_t m0 = __ballot(f0), m1 = __ballot(f1);
                const int nf0 = __popcll(m0), nf = nf0 + __popcll(m1);
                const uint64_t idle2 = __ballot(mode == kIdle);
                const int need = __popcll(idle2);
                const int q0 = __popcll(m0 & below), q1 = nf0 + __popcll(m1 & below);
                if (f0 && q0 < need) cand[q0] = (int32_t)sc0;
                if (f1 && q1 < need) cand[q1] = (int32_t)sc1;
                if (nf > need) {
                    if (f0 && q0 == need - 1) cut_at = sc0 + 1;
                    if (f1 && q1 == need - 1) cut_at = sc1 + 1;
                }
                __syncthreads();
                const int got = min(need, nf);
                if (mode == kIdle) {
                    const int r = __popcll(idle2 & below);
                    if (r < got) {
                        w = cand[r];
                        mode = kArrive;
                        is_start = true;
                        fresh = true;
                    }
                }
                cursor = (nf > need) ? cut_at : min(n, cursor + 2 * kWave);
            }

            // ---- 4. advance every walker by what its load returned
            bool claim = false, parked = false, push = false, bad = false;
            int32_t wait_on = lane, pushed = -1;
            if (!fresh) {
                if (mode == kDraw) {
                    w = v_col;
                    if (kh >= kMaxDraws) {
                        raise_err(p.err, kErrDrawOverflow, h);
                        bad = true;
                    } else {
                        st[h] = st_pack(w, kh + 1, (uint32_t)lane + 1, ep);
                        kh += 1;
                        ++s_draws;
                    }
                    mode = kArrive;
                    is_start = false;
                } else if (mode == kArrive) {
                    const uint32_t t = st_tag(v_st, ep);
                    if (t == kTagTree) {
                        if (is_start) {
                            mode = kIdle;
                        } else {
                            mode = kRetrace;   // path s..h joins the tree
                            x = s;
                        }
                    } else if (t == (uint32_t)lane + 1 && !is_start) {
                        // loop closed at w: pop the entries after w, resume at w
                        e = w;
                        ke = st_k(v_st, ep);
                        nbe = v_nb;
                        x = st_next(v_st);
                        stop_at = h;
                        mode = kRelease;
                    } else if (t == kTagFree) {
                        claim = true;
                    } else if (t <= (uint32_t)kWave) {
                        if (is_start) {
                            mode = kIdle;
                        } else {
                            parked = true;
                            wait_on = (int32_t)t - 1;
                        }
                    } else {
                        bad = true;   // a tag no walker of this wave can hold
                    }
                } else if (mode == kRetrace) {
                    const uint32_t k = st_k(v_st, ep);
                    const int32_t nx = st_next(v_st);
                    st[x] = st_pack(nx, k, kTagTree, ep);
                    if (y1b) atomicAdd(&y1b[x], (unsigned long long)k);
                    y1_local += k;
                    ++tree_local;
                    if (keep_q >= 0) {
                        if (p.next_out) p.next_out[(int64_t)keep_q * n + x] = nx;
                        if (p.draws_out) p.draws_out[(int64_t)keep_q * n + x] = (int32_t)k;
                    }
                    if (x == h) mode = kIdle;
                    else x = nx;
                } else if (mode == kRelease) {
                    const int32_t nx = st_next(v_st);
                    st[x] = st_pack(nx, st_k(v_st, ep), kTagFree, ep);
                    if (x < cursor) {
                        push = true;
                        pushed = x;
                    }
                    if (x == stop_at) {
                        h = e;
                        kh = ke;
                        nbh = nbe;
                        mode = kDraw;
                    } else {
                        x = nx;
                    }
                } else if (mode == kPopLoad) {
                    ke = st_k(v_st, ep);
                    nbe = v_nb;
                    x = st_next(v_st);
                    stop_at = h;
                    mode = kRelease;
                }
            }

            if (__ballot(bad)) {
                stop = true;
                break;
            }

            // ---- 5. claims of free nodes, deduplicated through an LDS table
            if (claim) claim_tbl[w & kClaimMask] = (uint8_t)lane;
            __syncthreads();
            const int winner = claim ? (int)claim_tbl[w & kClaimMask] : lane;
            const int32_t w_win = __shfl(w, winner, kWave);
            if (claim) {
                if (winner == lane) {
                    const uint32_t kw = st_k(v_st, ep);
                    st[w] = st_pack(st_current(v_st, ep) ? st_next(v_st) : -1, kw, (uint32_t)lane + 1, ep);
                    if (is_start) {
                        s = w;
                        is_start = false;
                    }
                    h = w;
                    kh = kw;
                    nbh = v_nb;
                    mode = kDraw;
                } else if (w_win == w) {
                    if (is_start) {
                        mode = kIdle;
                    } else {
                        parked = true;
                        wait_on = winner;
                    }
                }
                // otherwise a different node hashed to the same slot: retry
            }

            // ---- 6. rings of parked walkers are cycles of stack tops: pop them
            const uint64_t pk = __ballot(parked);
            if (__popcll(pk) >= 2) {
                const int f = parked ? wait_on : lane;
                int g = f;
#pragma unroll
                for (int r = 0; r < 6; ++r) g = __shfl(g, g, kWave);   // g = f^64(lane)
                mark[lane] = 0;
                __syncthreads();
                mark[g] = 1;
                __syncthreads();
                const bool on_cycle = parked && mark[lane] != 0;
                if (on_cycle) ent[f] = w;
                __syncthreads();
                if (on_cycle) {
                    e = ent[lane];
                    parked = false;
                    mode = (e == h) ? kDraw : kPopLoad;
                }
                const uint64_t cyc = __ballot(on_cycle);
                if (lane == 0 && cyc) ++s_pops;
            }

            // ---- 7. released nodes behind the scan go on the revisit list
            const uint64_t pm = __ballot(push);
            if (pm) {
                const int r = __popcll(pm & below);
                const int c = __popcll(pm);
                if (push && rev_n + r < kRevCap) rev[rev_n + r] = pushed;
                if (rev_n + c > kRevCap) {
                    overflow = true;
                    rev_n = kRevCap;
                } else {
                    rev_n += c;
                }
            }
            fresh = false;
            __syncthreads();   // stores and LDS writes visible to the next round
            if (lane == 0) ++s_iters;

            // ---- 8. the sample ends when every node is in the tree
            const uint64_t busy = __ballot(mode != kIdle);
            if (!busy && rev_n == 0 && cursor >= n) {
                const int64_t tc = wave_sum_i64(tree_local);
                if (tc == n) break;
                if (overflow) {
                    overflow = false;
                    cursor = 0;
                    if (lane == 0) ++s_rescans;
                } else {
                    if (lane == 0) raise_err(p.err, kErrInconsistent, (int32_t)tc);
                    stop = true;
                    break;
                }
            }
        }
        if (stop) break;
        const int64_t y1 = wave_sum_i64(y1_local);
        if (lane == 0) {
            if (p.y1_per_sample) p.y1_per_sample[smp] = y1;
            ++s_trees;
        }
    }
    if (lane == 0) p.slot_epoch[slot] = ep;
    const int64_t d = wave_sum_i64((int64_t)s_draws);
    if (lane == 0) {
        atomicAdd(&p.stats[kStatIters], s_iters);
        atomicAdd(&p.stats[kStatDraws], (unsigned long long)d);
        atomicAdd(&p.stats[kStatTrees], s_trees);
        atomicAdd(&p.stats[kStatPops], s_pops);
        atomicAdd(&p.stats[kStatRescans], s_rescans);
    }
}

// ----------------------------------------------------------------- launchers
hipError_t launch_wilson_lane(const WilsonParams &p, int64_t slots, hipStream_t s) {
    const int bs = 64;
    const int64_t grid = (slots + bs - 1) / bs;
    hipLaunchKernelGGL(wilson_lane_kernel, dim3((unsigned)grid), dim3(bs), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_wilson_wave(const WilsonParams &p, int64_t slots, hipStream_t s) {
    hipLaunchKernelGGL(wilson_wave_kernel, dim3((unsigned)slots), dim3(kWave), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
