// The wave-cooperative Wilson sample: 64 lanes of one wavefront run
// concurrent loop-erased walks of one sample (the algorithm is described in
// wilson.hip).  Included by the plain and the batched kernels.
#pragma once

#include "lap_device.h"

namespace lap {

constexpr int kWave = 64;
constexpr int kClaimBits = 11;
constexpr int kClaimMask = (1 << kClaimBits) - 1;
constexpr int kRevCap = 256;

enum : int32_t { kIdle = 0, kDraw = 1, kArrive = 2, kRetrace = 3, kRelease = 4, kPopLoad = 5 };

static __device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

static __device__ __forceinline__ int64_t block_of(int64_t sample, int32_t B, int64_t n_total) {
    return (sample * (int64_t)B) / n_total;
}

// ----------------------------------------------------------------- wave form
struct WaveShared {
    uint8_t claim_tbl[1 << kClaimBits];
    int32_t rev[kRevCap];
    int32_t cand[2 * kWave];
    int32_t ent[kWave];
    int32_t mark[kWave];
    int64_t cut_at;
};

// One Wilson sample run by the calling wavefront's 64 lanes (see the file
// header).  Returns false when the sample was abandoned (error or time limit;
// p.err says which); *y1_out receives the sample's total draws.
static __device__ bool wave_wilson_sample(const WaveSampleArgs &c, WaveShared &sh, int64_t *y1_out, WaveStats &ws) {
    const int lane = (int)threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t n = c.n;
    uint64_t *st = c.st;
    const uint32_t ep = c.ep;
    const int64_t sample = c.sample;
    if (lane == 0) {
        st[c.root] = st_pack(-1, 0, kTagTree, ep);
        if (c.keep_next) c.keep_next[c.root] = -1;
        if (c.keep_draws) c.keep_draws[c.root] = 0;
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
            int bad = (wall_clock64() - c.t0 > c.deadline) ? 2 : (err_set(c.err) ? 1 : 0);
            bad = __builtin_amdgcn_readfirstlane(bad);
            if (bad) {
                if (bad == 2) raise_err(c.err, kErrTimeout, 0);
                return false;
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
                    w = sh.rev[rev_n - 1 - r];
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
            const uint64_t r = philox_w0((uint64_t)sample, (uint64_t)h, kh, c.qid, c.k0, c.k1);
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
                         (mode == kDraw && (h < 0 || h >= n || ld_col < 0 || ld_col >= c.nnz));
        if (__ballot(oob)) {
            if (oob) raise_err(c.err, kErrInconsistent, -1);
            return false;
        }
        const int64_t sc0 = cursor + lane, sc1 = cursor + kWave + lane;
        const uint64_t v_st = (ld_st >= 0) ? st[ld_st] : 0ull;
        const uint64_t v_nb = (ld_nb >= 0) ? c.nbr[ld_nb] : 0ull;
        const int32_t v_col = (ld_col >= 0) ? c.col[ld_col] : 0;
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
            if (f0 && q0 < need) sh.cand[q0] = (int32_t)sc0;
            if (f1 && q1 < need) sh.cand[q1] = (int32_t)sc1;
            if (nf > need) {
                if (f0 && q0 == need - 1) sh.cut_at = sc0 + 1;
                if (f1 && q1 == need - 1) sh.cut_at = sc1 + 1;
            }
            __syncthreads();
            const int got = min(need, nf);
            if (mode == kIdle) {
                const int r = __popcll(idle2 & below);
                if (r < got) {
                    w = sh.cand[r];
                    mode = kArrive;
                    is_start = true;
                    fresh = true;
                }
            }
            cursor = (nf > need) ? sh.cut_at : min(n, cursor + 2 * kWave);
        }

        // ---- 4. advance every walker by what its load returned
        bool claim = false, parked = false, push = false, bad = false;
        int32_t wait_on = lane, pushed = -1;
        if (!fresh) {
            if (mode == kDraw) {
                w = v_col;
                if (kh >= kMaxDraws) {
                    raise_err(c.err, kErrDrawOverflow, h);
                    bad = true;
                } else {
                    st[h] = st_pack(w, kh + 1, (uint32_t)lane + 1, ep);
                    kh += 1;
                    ++ws.draws;
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
                if (c.y1b) atomicAdd(&c.y1b[x], (unsigned long long)k);
                y1_local += k;
                ++tree_local;
                if (c.keep_next) c.keep_next[x] = nx;
                if (c.keep_draws) c.keep_draws[x] = (int32_t)k;
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
            if (bad) raise_err(c.err, kErrInconsistent, -2);
            return false;
        }

        // ---- 5. claims of free nodes, deduplicated through an LDS table
        if (claim) sh.claim_tbl[w & kClaimMask] = (uint8_t)lane;
        __syncthreads();
        const int winner = claim ? (int)sh.claim_tbl[w & kClaimMask] : lane;
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
            sh.mark[lane] = 0;
            __syncthreads();
            sh.mark[g] = 1;
            __syncthreads();
            const bool on_cycle = parked && sh.mark[lane] != 0;
            if (on_cycle) sh.ent[f] = w;
            __syncthreads();
            if (on_cycle) {
                e = sh.ent[lane];
                parked = false;
                mode = (e == h) ? kDraw : kPopLoad;
            }
            const uint64_t cyc = __ballot(on_cycle);
            if (lane == 0 && cyc) ++ws.pops;
        }

        // ---- 7. released nodes behind the scan go on the revisit list
        const uint64_t pm = __ballot(push);
        if (pm) {
            const int r = __popcll(pm & below);
            const int cnt = __popcll(pm);
            if (push && rev_n + r < kRevCap) sh.rev[rev_n + r] = pushed;
            if (rev_n + cnt > kRevCap) {
                overflow = true;
                rev_n = kRevCap;
            } else {
                rev_n += cnt;
            }
        }
        fresh = false;
        __syncthreads();   // stores and LDS writes visible to the next round
        if (lane == 0) ++ws.iters;

        // ---- 8. the sample ends when every node is in the tree
        const uint64_t busy = __ballot(mode != kIdle);
        if (!busy && rev_n == 0 && cursor >= n) {
            const int64_t tc = wave_sum_i64(tree_local);
            if (tc == n) break;
            if (overflow) {
                overflow = false;
                cursor = 0;
                if (lane == 0) ++ws.rescans;
            } else {
                if (lane == 0) raise_err(c.err, kErrInconsistent, (int32_t)tc);
                return false;
            }
        }
    }
    *y1_out = wave_sum_i64(y1_local);
    return true;
}

static __device__ void flush_wave_stats(const WaveStats &ws, unsigned long long *stats) {
    const int64_t d = wave_sum_i64((int64_t)ws.draws);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[kStatIters], ws.iters);
        atomicAdd(&stats[kStatDraws], (unsigned long long)d);
        atomicAdd(&stats[kStatTrees], ws.trees);
        atomicAdd(&stats[kStatPops], ws.pops);
        atomicAdd(&stats[kStatRescans], ws.rescans);
    }
}

}  // namespace lap
