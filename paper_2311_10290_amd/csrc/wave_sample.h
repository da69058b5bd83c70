// The wave-cooperative Wilson sample: the 64 lanes of one wavefront run
// concurrent loop-erased walks of one sample (protocol in wilson.hip).
// Included by the plain and the batched kernels.
//
// Each walker keeps its current path -- node ids and their draw counts -- in
// a small LDS stack, so closing a loop, popping a cycle and joining the tree
// only write state words (no re-reads), and a draw needs no store at all:
// other walkers only look at a node's tag, which the claim already wrote.  A
// path longer than the stack, or a node with more than 255 draws, moves the
// walker to memory mode: the stack is written out as next/draw words and the
// walk continues by storing every draw and following next pointers.
#pragma once

#include "lap_device.h"

namespace lap {

constexpr int kWave = 64;
constexpr int kClaimBits = 11;
constexpr int kClaimMask = (1 << kClaimBits) - 1;
constexpr int kRevCap = 256;
constexpr int kStackDepth = 12;
constexpr uint32_t kStackMaxK = 255;
constexpr int kScanChunks = 2;

enum : int32_t {
    kIdle = 0,
    kDraw = 1,      // draw at the head h
    kArrive = 2,    // look at the target w (also: parked, waiting on w)
    kRetrace = 3,   // memory mode: mark the path s..h as tree, one node per round
    kRelease = 4,   // memory mode: free the popped nodes x..stop_at, one per round
    kPopLoad = 5,   // memory mode: load the entry node e of a popped cycle
    kNbLoad = 6     // stack mode: load the adjacency record of the resumed head
};

static __device__ __forceinline__ int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

static __device__ __forceinline__ int64_t block_of(int64_t sample, int32_t B, int64_t n_total) {
    return (sample * (int64_t)B) / n_total;
}

struct WaveShared {
    int32_t stk_node[kStackDepth][kWave];
    uint8_t stk_k[kStackDepth][kWave];
    uint8_t claim_tbl[1 << kClaimBits];
    int32_t rev[kRevCap];
    int32_t cand_node[kWave];
    uint64_t cand_st[kWave];
    uint64_t cand_nb[kWave];
    int32_t ent[kWave];
    int32_t mark[kWave];
    int64_t cut_at;
};

// LDS ordering inside the single-wave workgroup: wait for this wave's LDS
// operations, no wait on global memory
static __device__ __forceinline__ void wave_lds_sync() {
    __builtin_amdgcn_s_waitcnt(0xC07F);   // lgkmcnt(0)
    __builtin_amdgcn_wave_barrier();
}

// One Wilson sample run by the calling wavefront.  Returns false when the
// sample was abandoned (error or time limit; c.err says which); *y1_out is
// the sample's total number of draws.
//
// A round of the loop: (1) the drawing walkers load their drawn column entry
// (read-only data); (2) a workgroup fence makes the previous round's state
// stores visible -- their completion overlaps the column loads; (3) every
// arriving walker loads its target's state word and adjacency record, and
// the scan loads the next candidate starts; (4) walkers act on what they
// loaded; walkers that are idle now take free candidates from this round's
// scan and claim them at once.
template <bool ARCS = false>
static __device__ bool wave_wilson_sample(const WaveSampleArgs &c, WaveShared &sh, int64_t *y1_out, WaveStats &ws) {
    const int lane = (int)threadIdx.x;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t n = c.n;
    uint64_t *st = c.st;
    const uint32_t ep = c.ep;
    const int64_t sample = c.sample;
    const uint32_t me = (uint32_t)lane + 1;
    if (lane == 0) {
        st[c.root] = st_pack(-1, 0, kTagTree, ep);
        if (c.keep_next) c.keep_next[c.root] = -1;
        if (c.keep_draws) c.keep_draws[c.root] = 0;
    }

    // the scan visits positions 0..n-1; position p is node (p + scan_offset) mod n
    // (any offset gives the same counts: a schedule knob for race tests)
    int64_t cursor = 0;        // next scan position (wave-uniform)
    const int64_t off = c.scan_offset;
    auto node_at = [&](int64_t p) -> int64_t { const int64_t q = p + off; return q >= n ? q - n : q; };
    auto pos_of = [&](int64_t x) -> int64_t { const int64_t q = x - off; return q < 0 ? q + n : q; };
    int rev_n = 0;             // entries in rev[] (wave-uniform)
    bool overflow = false;     // rev[] overflowed: rescan needed (wave-uniform)
    int64_t tree_local = (lane == 0) ? 1 : 0;
    int64_t y1_local = 0;
    int mode = kIdle;
    bool is_start = false;     // the ARRIVE target is a start candidate
    bool fresh = false;        // wrote its stack out this round: arrive next round
    bool mem = false;          // memory mode (path not on the LDS stack)
    int depth = 0;             // stack entries (stack mode)
    int32_t s = -1, h = -1, w = -1, x = -1, stop_at = -1, e = -1;
    uint32_t kh = 0, ke = 0;
    uint64_t nbh = 0, nbe = 0;
    uint64_t nbw = 0;          // arc form: the target's adjacency record, when nbw_ok
    bool nbw_ok = false;
    uint64_t it = 0;

    // write the stack out as path words: entry j points to entry j+1, the top
    // to top_next (memory mode from here on)
    auto flush_stack = [&](int32_t top_next, uint32_t top_k) {
        for (int j = 0; j < depth; ++j) {
            const int32_t node = sh.stk_node[j][lane];
            const bool top = j + 1 == depth;
            const int32_t nx = top ? top_next : sh.stk_node[j + 1][lane];
            st[node] = st_pack(nx, top ? top_k : (uint32_t)sh.stk_k[j][lane], me, ep);
        }
        depth = 0;
        mem = true;
    };
    auto push_round = [&](bool pu, int32_t node) {
        const uint64_t pm = __ballot(pu);
        if (pm) {
            const int r = __popcll(pm & below);
            const int cnt = __popcll(pm);
            if (pu && rev_n + r < kRevCap) sh.rev[rev_n + r] = node;
            if (rev_n + cnt > kRevCap) {
                overflow = true;
                rev_n = kRevCap;
            } else {
                rev_n += cnt;
            }
        }
    };

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
        // ---- R1. read-only loads: drawn column entries, resumed heads' adjacency
        int64_t la_col = -1, la_nb1 = -1;
        if (mode == kDraw) {
            const uint64_t r = philox_w0((uint64_t)sample, (uint64_t)h, kh, c.qid, c.k0, c.k1);
            la_col = nbr_off(nbh) + (int64_t)pick_below(r, nbr_deg(nbh));
        } else if (mode == kNbLoad) {
            la_nb1 = h;
        }
        {
            // every index must stay inside the graph; anything else is a bug
            // and stops the kernel instead of touching memory out of bounds
            const bool oob = (mode == kDraw && (h < 0 || h >= n || la_col < 0 || la_col >= c.nnz)) ||
                             (mode == kNbLoad && (la_nb1 < 0 || la_nb1 >= n));
            if (__ballot(oob)) {
                if (oob) raise_err(c.err, kErrInconsistent, -1);
                return false;
            }
        }
        int32_t a_col = 0;
        uint64_t a_nbw = 0;
        if constexpr (ARCS) {
            if (la_col >= 0) {
                const ulonglong2 av = c.arcs[la_col];
                a_col = (int32_t)av.x;
                a_nbw = av.y;
            }
        } else {
            a_col = (la_col >= 0) ? c.col[la_col] : 0;
        }
        const uint64_t a_nb1 = (la_nb1 >= 0) ? c.nbr[la_nb1] : 0ull;

        // ---- fence: the previous round's stores and LDS writes are visible
        __syncthreads();

        // ---- 1. idle walkers take released nodes the scan has passed
        const uint64_t idle = __ballot(mode == kIdle);
        const int n_idle = __popcll(idle);
        if (n_idle > 0) {
            const int take = min(n_idle, rev_n);
            if (mode == kIdle) {
                const int r = __popcll(idle & below);
                if (r < take) {
                    w = sh.rev[rev_n - 1 - r];
                    nbw_ok = false;
                    mode = kArrive;
                    is_start = true;
                }
            }
            rev_n -= take;
        }

        // ---- 2. finish draws: the drawn neighbour becomes the next target
        bool bad = false;
        if (mode == kDraw) {
            w = a_col;
            if constexpr (ARCS) {
                nbw = a_nbw;
                nbw_ok = true;
            }
            if (kh >= kMaxDraws) {
                raise_err(c.err, kErrDrawOverflow, h);
                bad = true;
            } else if (mem) {
                st[h] = st_pack(w, kh + 1, me, ep);
                kh += 1;
            } else if (kh + 1 > kStackMaxK) {
                flush_stack(w, kh + 1);
                kh += 1;
                fresh = true;      // arrive next round, once the words are visible
            } else {
                kh += 1;
                sh.stk_k[depth - 1][lane] = (uint8_t)kh;
            }
            ++ws.draws;
            mode = kArrive;
            is_start = false;
        } else if (mode == kNbLoad) {
            nbh = a_nb1;
            mode = kDraw;
        }

        // ---- R2. state loads: arriving walkers, memory-mode walkers, the scan
        const bool arriving = (mode == kArrive) && !fresh;
        int64_t lb_st = -1, lb_nb = -1;
        if (arriving) {
            lb_st = w;
            lb_nb = (ARCS && nbw_ok) ? -1 : w;
        } else if (mode == kRetrace || mode == kRelease) {
            lb_st = x;
        } else if (mode == kPopLoad) {
            lb_st = e;
            lb_nb = e;
        }
        if ((lb_st >= 0 && lb_st >= n) || (lb_nb >= 0 && lb_nb >= n) ||
            ((arriving || mode == kRetrace || mode == kRelease || mode == kPopLoad) && lb_st < 0))
            bad = true;
        if (__ballot(bad)) {
            if (bad) raise_err(c.err, kErrInconsistent, -2);
            return false;
        }
        const int scan_chunks = (cursor < n) ? (n_idle > 0 ? kScanChunks : 1) : 0;   // wave-uniform
        uint64_t v_st = (lb_st >= 0) ? st[lb_st] : 0ull;
        uint64_t v_nb = (lb_nb >= 0) ? c.nbr[lb_nb] : 0ull;
        uint64_t sc_st[kScanChunks], sc_nb[kScanChunks];
#pragma unroll
        for (int q = 0; q < kScanChunks; ++q) {
            const int64_t sc = cursor + q * kWave + lane;
            const bool ld = q < scan_chunks && sc < n;
            const int64_t nd = ld ? node_at(sc) : 0;
            sc_st[q] = ld ? st[nd] : 0ull;
            sc_nb[q] = ld ? c.nbr[nd] : 0ull;
        }

        // ---- C. advance every walker by what its loads returned
        if constexpr (ARCS) {
            if (arriving) {
                if (nbw_ok) {
                    v_nb = nbw;
                } else {
                    nbw = v_nb;
                    nbw_ok = true;
                }
            }
        }
        bool claim = false, parked = false, push = false;
        int32_t wait_on = lane, pushed = -1;
        int rel_lo = 0, rel_hi = 0;     // stack entries to release this round
        if (arriving) {
            const uint32_t t = st_tag(v_st, ep);
            if (t == kTagTree) {
                if (is_start) {
                    mode = kIdle;
                } else if (mem) {
                    mode = kRetrace;   // path s..h joins the tree, one node per round
                    x = s;
                } else {
                    // the whole path joins the tree now
                    for (int j = 0; j < depth; ++j) {
                        const int32_t node = sh.stk_node[j][lane];
                        const uint32_t k = sh.stk_k[j][lane];
                        const int32_t nx = (j + 1 < depth) ? sh.stk_node[j + 1][lane] : w;
                        st[node] = st_pack(nx, k, kTagTree, ep);
                        if (c.y1b && k > 1) atomicAdd(&c.y1b[node], (unsigned long long)(k - 1));
                        y1_local += k;
                        if (c.keep_next) c.keep_next[node] = nx;
                        if (c.keep_draws) c.keep_draws[node] = (int32_t)k;
                    }
                    tree_local += depth;
                    depth = 0;
                    mode = kIdle;
                }
            } else if (t == me && !is_start) {
                // loop closed at w: pop the entries after w, resume at w
                if (mem) {
                    e = w;
                    ke = st_k(v_st, ep);
                    nbe = v_nb;
                    x = st_next(v_st);
                    stop_at = h;
                    mode = kRelease;
                } else {
                    int p = -1;
                    for (int j = 0; j < depth; ++j)
                        if (sh.stk_node[j][lane] == w) p = j;
                    if (p < 0) {
                        bad = true;
                    } else {
                        rel_lo = p + 1;
                        rel_hi = depth;
                        depth = p + 1;
                        h = w;
                        kh = sh.stk_k[p][lane];
                        nbh = v_nb;
                        mode = kDraw;
                    }
                }
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
            if (c.y1b && k > 1) atomicAdd(&c.y1b[x], (unsigned long long)(k - 1));
            y1_local += k;
            ++tree_local;
            if (c.keep_next) c.keep_next[x] = nx;
            if (c.keep_draws) c.keep_draws[x] = (int32_t)k;
            if (x == h) {
                mode = kIdle;
                mem = false;
            } else {
                x = nx;
            }
        } else if (mode == kRelease) {
            const int32_t nx = st_next(v_st);
            st[x] = st_pack(nx, st_k(v_st, ep), kTagFree, ep);
            push = true;
            pushed = x;
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
        if (__ballot(bad)) {
            if (bad) raise_err(c.err, kErrInconsistent, -3);
            return false;
        }

        // ---- scan: walkers idle now take FREE candidates and claim them
        if (scan_chunks > 0) {
            const uint64_t idle2 = __ballot(mode == kIdle);
            const int need = __popcll(idle2);
            if (need > 0) {
                uint64_t m[kScanChunks];
                int nf = 0;
#pragma unroll
                for (int q = 0; q < kScanChunks; ++q) {
                    const int64_t sc = cursor + q * kWave + lane;
                    m[q] = __ballot(q < scan_chunks && sc < n && st_tag(sc_st[q], ep) == kTagFree);
                    nf += __popcll(m[q]);
                }
                int base = 0;
#pragma unroll
                for (int q = 0; q < kScanChunks; ++q) {
                    const bool f = (m[q] >> lane) & 1ull;
                    const int qq = base + __popcll(m[q] & below);
                    const int64_t sc = cursor + q * kWave + lane;
                    if (f && qq < need) {
                        sh.cand_node[qq] = (int32_t)node_at(sc);
                        sh.cand_st[qq] = sc_st[q];
                        sh.cand_nb[qq] = sc_nb[q];
                    }
                    if (f && qq == need - 1 && nf > need) sh.cut_at = sc + 1;
                    base += __popcll(m[q]);
                }
                wave_lds_sync();
                const int got = min(need, nf);
                if (mode == kIdle) {
                    const int r = __popcll(idle2 & below);
                    if (r < got) {
                        w = sh.cand_node[r];
                        v_st = sh.cand_st[r];
                        v_nb = sh.cand_nb[r];
                        nbw = v_nb;
                        nbw_ok = true;
                        mode = kArrive;
                        is_start = true;
                        claim = true;
                    }
                }
                cursor = (nf > need) ? sh.cut_at : min(n, cursor + (int64_t)scan_chunks * kWave);
            }
        }

        // ---- claims of free nodes, deduplicated through an LDS table
        if (claim) sh.claim_tbl[w & kClaimMask] = (uint8_t)lane;
        wave_lds_sync();
        const int winner = claim ? (int)sh.claim_tbl[w & kClaimMask] : lane;
        const int32_t w_win = __shfl(w, winner, kWave);
        if (claim) {
            if (winner == lane) {
                const uint32_t kw = st_k(v_st, ep);
                if (is_start) {
                    s = w;
                    is_start = false;
                    mem = false;
                    depth = 0;
                }
                if (!mem && (depth == kStackDepth || kw > kStackMaxK)) flush_stack(w, (uint32_t)sh.stk_k[depth > 0 ? depth - 1 : 0][lane]);
                st[w] = st_pack(-1, kw, me, ep);
                if (!mem) {
                    sh.stk_node[depth][lane] = w;
                    sh.stk_k[depth][lane] = (uint8_t)kw;
                    ++depth;
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
            // (a start candidate that lost this way is looked at again next round)
        }

        // ---- rings of parked walkers are cycles of stack tops: pop them
        const uint64_t pk = __ballot(parked);
        if (__popcll(pk) >= 2) {
            const int f = parked ? wait_on : lane;
            int g = f;
#pragma unroll
            for (int r = 0; r < 6; ++r) g = __shfl(g, g, kWave);   // g = f^64(lane)
            sh.mark[lane] = 0;
            wave_lds_sync();
            sh.mark[g] = 1;
            wave_lds_sync();
            const bool on_cycle = parked && sh.mark[lane] != 0;
            if (on_cycle) sh.ent[f] = w;
            wave_lds_sync();
            if (on_cycle) {
                e = sh.ent[lane];
                parked = false;
                if (mem) {
                    mode = (e == h) ? kDraw : kPopLoad;
                } else {
                    int p = -1;
                    for (int j = 0; j < depth; ++j)
                        if (sh.stk_node[j][lane] == e) p = j;
                    if (p < 0) {
                        bad = true;
                    } else {
                        rel_lo = p + 1;
                        rel_hi = depth;
                        depth = p + 1;
                        if (e != h) {
                            h = e;
                            kh = sh.stk_k[p][lane];
                            mode = kNbLoad;
                        } else {
                            mode = kDraw;
                        }
                    }
                }
            }
            const uint64_t cyc = __ballot(on_cycle);
            if (lane == 0 && cyc) ++ws.pops;
            if (__ballot(bad)) {
                if (bad) raise_err(c.err, kErrInconsistent, -4);
                return false;
            }
        }

        // ---- released nodes: free words; those behind the scan go on the revisit list
        push_round(push && pos_of(pushed) < cursor, pushed);
        if (__ballot(rel_hi > rel_lo)) {
            for (int j = 0; j < kStackDepth; ++j) {
                const bool act = j >= rel_lo && j < rel_hi;
                int32_t node = -1;
                if (act) {
                    node = sh.stk_node[j][lane];
                    st[node] = st_pack(-1, sh.stk_k[j][lane], kTagFree, ep);
                }
                push_round(act && pos_of(node) < cursor, node);
            }
        }
        fresh = false;
        wave_lds_sync();
        if (lane == 0) {
            ++ws.iters;
            ws.idle += (unsigned long long)n_idle;
            ws.parked += (unsigned long long)__popcll(pk);
        }

        // ---- the sample ends when every node is in the tree
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
    // leave the sample's stores visible before the slot is reused
    __syncthreads();
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
        atomicAdd(&stats[kStatIdleLanes], ws.idle);
        atomicAdd(&stats[kStatParkedLanes], ws.parked);
    }
}

}  // namespace lap
