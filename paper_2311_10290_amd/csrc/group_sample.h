// The workgroup-cooperative Wilson sample: W wavefronts -- 64*W walkers --
// run one sample together.  The walker protocol is the wave form's
// (wave_sample.h): claims by tag, loops closed on the walker's own LDS path
// stack, parking on another walker's path, rings of parked walkers popped as
// one cycle of stack tops, starts from a coalesced scan and a revisit list.
// Only the exchanges between walkers change: they go through LDS across
// workgroup barriers instead of wave ballots and shuffles.
//
// Used when a launch has too few samples to fill the chip with one wave per
// sample (a large graph with a few hundred trees): the workgroup form keeps
// 64*W dependent-load chains of one sample in flight.
//
// Every barrier below is executed by all threads in every round; the loop
// exits only on workgroup-uniform values read after a barrier, so the
// barrier sequence is the same for every wave.  A thread that detects an
// inconsistency raises the error, keeps its indices in bounds for the rest
// of the round, and the whole workgroup returns at the next round's fence.
#pragma once

#include <type_traits>

#include "wave_sample.h"

namespace lap {

constexpr int kGroupRevCap = 1024;
constexpr int kGroupScanChunks = 1;

// claim table: about 32 slots per walker (a claim that shares its slot with
// another node's retries next round), entries wide enough for a walker id
template <int W>
struct GroupClaim {
    static constexpr int kBits = W <= 2 ? 12 : 13;
    static constexpr int kMask = (1 << kBits) - 1;
    using Entry = typename std::conditional<kWave * W <= 256, uint8_t, uint16_t>::type;
};

template <int W>
struct GroupShared {
    static constexpr int NW = kWave * W;
    int32_t stk_node[kStackDepth][NW];
    uint8_t stk_k[kStackDepth][NW];
    typename GroupClaim<W>::Entry claim_tbl[1 << GroupClaim<W>::kBits];
    int32_t claim_w[NW];
    int32_t rev[kGroupRevCap];
    int32_t cand_node[NW];
    uint64_t cand_st[NW];
    uint64_t cand_nb[NW];
    int32_t f[NW];         // wait-for: the walker a parked walker waits on, else itself
    int32_t tw[NW];        // the node a parked walker waits at
    int32_t ent[NW];       // entry node handed to a walker on a popped ring, else -1
    int32_t jmp[2][NW];
    uint8_t mark[NW];
    int32_t cnt_idle[W];   // idle walkers per wave at the end of the round
    int32_t cnt_idle2[W];  // idle walkers per wave after acting (scan takers)
    int32_t cnt_free[kGroupScanChunks][W];
    int32_t cnt_parked[W];
    int64_t part[W];       // per-wave tree counts (and the final draw total)
    int32_t push_cnt[2];   // revisit-list appends of the round, by round parity
    int32_t ovf[2];        // revisit-list overflow of the round, by round parity
    int32_t flag[2];       // abort request of the round (1 error, 2 time limit), by parity
    int64_t cut_at;
};

template <int W, bool ARCS = false>
static __device__ bool group_wilson_sample(const WaveSampleArgs &c, GroupShared<W> &sh, int64_t *y1_out,
                                           WaveStats &ws) {
    constexpr int NW = kWave * W;
    constexpr int kLogNW = W == 1 ? 6 : W == 2 ? 7 : W == 4 ? 8 : 9;
    static_assert(NW <= (int)kMaxWalkers && (NW & (NW - 1)) == 0, "walkers per sample");
    const int tid = (int)threadIdx.x;
    const int wave = tid >> 6, lane = tid & (kWave - 1);
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t n = c.n;
    uint64_t *st = c.st;
    const uint32_t ep = c.ep;
    const int64_t sample = c.sample;
    const uint32_t me = (uint32_t)tid + 1;
    if (tid == 0) {
        st[c.root] = st_pack(-1, 0, kTagTree, ep);
        if (c.keep_next) c.keep_next[c.root] = -1;
        if (c.keep_draws) c.keep_draws[c.root] = 0;
        sh.push_cnt[0] = sh.push_cnt[1] = 0;
        sh.ovf[0] = sh.ovf[1] = 0;
        sh.flag[0] = sh.flag[1] = 0;
    }
    if (lane == 0) {
        sh.cnt_idle[wave] = kWave;
        sh.part[wave] = 0;
    }

    const int64_t off = c.scan_offset;
    auto node_at = [&](int64_t p) -> int64_t { const int64_t q = p + off; return q >= n ? q - n : q; };
    auto pos_of = [&](int64_t x) -> int64_t { const int64_t q = x - off; return q < 0 ? q + n : q; };
    // workgroup-uniform copies, updated identically by every thread
    int64_t cursor = 0;
    int rev_n = 0;
    bool overflow = false;
    // per walker
    int64_t tree_local = (tid == 0) ? 1 : 0;
    int64_t y1_local = 0;
    int mode = kIdle;
    bool is_start = false, fresh = false, mem = false;
    int depth = 0;
    int32_t s = -1, h = -1, w = -1, x = -1, stop_at = -1, e = -1;
    uint32_t kh = 0, ke = 0;
    uint64_t nbh = 0, nbe = 0;
    uint64_t nbw = 0;          // arc form: the target's adjacency record, when nbw_ok
    bool nbw_ok = false;
    uint64_t it = 0;
    bool done = false;

    auto flush_stack = [&](int32_t top_next, uint32_t top_k) {
        for (int j = 0; j < depth; ++j) {
            const int32_t node = sh.stk_node[j][tid];
            const bool top = j + 1 == depth;
            const int32_t nx = top ? top_next : sh.stk_node[j + 1][tid];
            st[node] = st_pack(nx, top ? top_k : (uint32_t)sh.stk_k[j][tid], me, ep);
        }
        depth = 0;
        mem = true;
    };

    while (true) {
        ++it;
        const int par = (int)(it & 1);
        // the time limit, decided by one thread and acted on after the next fence
        if ((it & 255) == 0 && tid == 0 && wall_clock64() - c.t0 > c.deadline) sh.flag[par] = 2;
        if ((it & 255) == 0 && tid == 0 && err_set(c.err)) sh.flag[par] = 1;
        bool bad = false;

        // ---- R1. read-only loads: drawn column entries, resumed heads' adjacency
        int64_t la_col = -1, la_nb1 = -1;
        if (mode == kDraw) {
            const uint64_t r = philox_w0((uint64_t)sample, (uint64_t)h, kh, c.qid, c.k0, c.k1);
            la_col = nbr_off(nbh) + (int64_t)pick_below(r, nbr_deg(nbh));
            if (h < 0 || h >= n || la_col < 0 || la_col >= c.nnz) bad = true;
        } else if (mode == kNbLoad) {
            la_nb1 = h;
            if (la_nb1 < 0 || la_nb1 >= n) bad = true;
        }
        if (bad) {
            la_col = la_nb1 = -1;
            raise_err(c.err, kErrInconsistent, -1);
            sh.flag[par] = 1;
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

        // ==== B1: the previous round's stores, LDS writes and counters are visible
        __syncthreads();

        // ---- workgroup-uniform bookkeeping from the previous round
        {
            const int fl = sh.flag[par ^ 1];
            if (fl) {
                if (fl == 2 && tid == 0) raise_err(c.err, kErrTimeout, 0);
                return false;
            }
        }
        int total_idle = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) total_idle += sh.cnt_idle[v];
        {
            const int pc = sh.push_cnt[par ^ 1];
            const int room = kGroupRevCap - rev_n;
            rev_n += pc < room ? pc : room;
            if (pc > room || sh.ovf[par ^ 1]) overflow = true;
        }
        if (total_idle == NW && rev_n == 0 && cursor >= n) {
            int64_t tc = 0;
#pragma unroll
            for (int v = 0; v < W; ++v) tc += sh.part[v];
            if (tc == n) {
                done = true;
            } else if (overflow) {
                overflow = false;
                cursor = 0;
                if (tid == 0) ++ws.rescans;
            } else {
                if (tid == 0) raise_err(c.err, kErrInconsistent, (int32_t)tc);
                return false;
            }
        }
        if (done) break;

        // ---- 1. idle walkers take released nodes the scan has passed
        const uint64_t idle_m = __ballot(mode == kIdle);
        {
            int pre = 0;
#pragma unroll
            for (int v = 0; v < W; ++v) pre += (v < wave) ? sh.cnt_idle[v] : 0;
            const int take = min(total_idle, rev_n);
            if (mode == kIdle) {
                const int r = pre + __popcll(idle_m & below);
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
                fresh = true;
            } else {
                kh += 1;
                sh.stk_k[depth - 1][tid] = (uint8_t)kh;
            }
            ++ws.draws;
            mode = kArrive;
            is_start = false;
        } else if (mode == kNbLoad) {
            nbh = a_nb1;
            mode = kDraw;
        }

        // ---- R2. state loads: arriving walkers, memory-mode walkers, the scan
        const bool arriving = (mode == kArrive) && !fresh && !bad;
        int64_t lb_st = -1, lb_nb = -1;
        if (arriving) {
            lb_st = w;
            lb_nb = (ARCS && nbw_ok) ? -1 : w;
        } else if (!bad && (mode == kRetrace || mode == kRelease)) {
            lb_st = x;
        } else if (!bad && mode == kPopLoad) {
            lb_st = e;
            lb_nb = e;
        }
        if (lb_st >= n || lb_nb >= n ||
            ((arriving || mode == kRetrace || mode == kRelease || mode == kPopLoad) && !bad && lb_st < 0)) {
            bad = true;
            lb_st = lb_nb = -1;
        }
        const int scan_chunks = (cursor < n) ? (total_idle > 0 ? kGroupScanChunks : 1) : 0;
        uint64_t v_st = (lb_st >= 0) ? st[lb_st] : 0ull;
        uint64_t v_nb = (lb_nb >= 0) ? c.nbr[lb_nb] : 0ull;
        uint64_t sc_st[kGroupScanChunks], sc_nb[kGroupScanChunks];
#pragma unroll
        for (int q = 0; q < kGroupScanChunks; ++q) {
            const int64_t sc = cursor + q * NW + tid;
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
        int32_t wait_on = tid, pushed = -1;
        int rel_lo = 0, rel_hi = 0;
        const bool act = !bad;
        if (act && arriving) {
            const uint32_t t = st_tag(v_st, ep);
            if (t == kTagTree) {
                if (is_start) {
                    mode = kIdle;
                } else if (mem) {
                    mode = kRetrace;
                    x = s;
                } else {
                    for (int j = 0; j < depth; ++j) {
                        const int32_t node = sh.stk_node[j][tid];
                        const uint32_t k = sh.stk_k[j][tid];
                        const int32_t nx = (j + 1 < depth) ? sh.stk_node[j + 1][tid] : w;
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
                        if (sh.stk_node[j][tid] == w) p = j;
                    if (p < 0) {
                        bad = true;
                    } else {
                        rel_lo = p + 1;
                        rel_hi = depth;
                        depth = p + 1;
                        h = w;
                        kh = sh.stk_k[p][tid];
                        nbh = v_nb;
                        mode = kDraw;
                    }
                }
            } else if (t == kTagFree) {
                claim = true;
            } else if (t <= (uint32_t)NW) {
                if (is_start) {
                    mode = kIdle;
                } else {
                    parked = true;
                    wait_on = (int32_t)t - 1;
                }
            } else {
                bad = true;
            }
        } else if (act && mode == kRetrace) {
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
        } else if (act && mode == kRelease) {
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
        } else if (act && mode == kPopLoad) {
            ke = st_k(v_st, ep);
            nbe = v_nb;
            x = st_next(v_st);
            stop_at = h;
            mode = kRelease;
        }
        if (bad) {
            // stop acting: the workgroup returns at the next fence
            claim = parked = push = false;
            rel_lo = rel_hi = 0;
            if (mode != kIdle) mode = kArrive;
            fresh = true;
            raise_err(c.err, kErrInconsistent, -3);
            sh.flag[par] = 1;
        }

        // ---- scan, part 1: count walkers idle now and free candidates, per wave
        const uint64_t idle2_m = __ballot(mode == kIdle);
        uint64_t fm[kGroupScanChunks];
#pragma unroll
        for (int q = 0; q < kGroupScanChunks; ++q) {
            const int64_t sc = cursor + q * NW + tid;
            fm[q] = __ballot(q < scan_chunks && sc < n && st_tag(sc_st[q], ep) == kTagFree);
        }
        if (lane == 0) {
            sh.cnt_idle2[wave] = __popcll(idle2_m);
#pragma unroll
            for (int q = 0; q < kGroupScanChunks; ++q) sh.cnt_free[q][wave] = __popcll(fm[q]);
        }

        // ==== B2
        __syncthreads();
        if (tid == 0) {
            // this slot's appends were read after the fence; it takes the next round's
            sh.push_cnt[par ^ 1] = 0;
            sh.ovf[par ^ 1] = 0;
        }

        // ---- scan, part 2: the first `need` free candidates in position order
        int need = 0, pre_idle2 = 0, nf = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) {
            need += sh.cnt_idle2[v];
            pre_idle2 += (v < wave) ? sh.cnt_idle2[v] : 0;
        }
        const bool scan_take = scan_chunks > 0 && need > 0;
        if (scan_take) {
            int base = 0;
#pragma unroll
            for (int q = 0; q < kGroupScanChunks; ++q) {
                int pre = 0, tot = 0;
#pragma unroll
                for (int v = 0; v < W; ++v) {
                    tot += sh.cnt_free[q][v];
                    pre += (v < wave) ? sh.cnt_free[q][v] : 0;
                }
                const bool f = (fm[q] >> lane) & 1ull;
                const int qq = base + pre + __popcll(fm[q] & below);
                const int64_t sc = cursor + q * NW + tid;
                if (f && qq < need) {
                    sh.cand_node[qq] = (int32_t)node_at(sc);
                    sh.cand_st[qq] = sc_st[q];
                    sh.cand_nb[qq] = sc_nb[q];
                }
                base += tot;
            }
            nf = base;
            base = 0;
#pragma unroll
            for (int q = 0; q < kGroupScanChunks; ++q) {
                int pre = 0, tot = 0;
#pragma unroll
                for (int v = 0; v < W; ++v) {
                    tot += sh.cnt_free[q][v];
                    pre += (v < wave) ? sh.cnt_free[q][v] : 0;
                }
                const bool f = (fm[q] >> lane) & 1ull;
                const int qq = base + pre + __popcll(fm[q] & below);
                if (f && qq == need - 1 && nf > need) sh.cut_at = cursor + q * NW + tid + 1;
                base += tot;
            }
        }

        // ==== B3
        __syncthreads();

        // ---- scan, part 3: walkers idle now take the candidates and claim them
        if (scan_take) {
            const int got = min(need, nf);
            if (mode == kIdle) {
                const int r = pre_idle2 + __popcll(idle2_m & below);
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
            cursor = (nf > need) ? sh.cut_at : min(n, cursor + (int64_t)scan_chunks * NW);
        }
        if (claim) {
            sh.claim_tbl[w & GroupClaim<W>::kMask] = (typename GroupClaim<W>::Entry)tid;
            sh.claim_w[tid] = w;
        }

        // ==== B4
        __syncthreads();

        // ---- claims of free nodes, deduplicated through the LDS table
        if (claim) {
            const int winner = (int)sh.claim_tbl[w & GroupClaim<W>::kMask];
            const int32_t w_win = sh.claim_w[winner];
            if (winner == tid) {
                const uint32_t kw = st_k(v_st, ep);
                if (is_start) {
                    s = w;
                    is_start = false;
                    mem = false;
                    depth = 0;
                }
                if (!mem && (depth == kStackDepth || kw > kStackMaxK))
                    flush_stack(w, (uint32_t)sh.stk_k[depth > 0 ? depth - 1 : 0][tid]);
                st[w] = st_pack(-1, kw, me, ep);
                if (!mem) {
                    sh.stk_node[depth][tid] = w;
                    sh.stk_k[depth][tid] = (uint8_t)kw;
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
            // otherwise a different node hashed to the same slot: retry next round
        }
        sh.f[tid] = parked ? wait_on : tid;
        sh.tw[tid] = w;
        const uint64_t pk = __ballot(parked);
        if (lane == 0) sh.cnt_parked[wave] = __popcll(pk);

        // ==== B5
        __syncthreads();

        // ---- rings of parked walkers: pointer jumping by wave 0 over all walkers
        int total_parked = 0;
#pragma unroll
        for (int v = 0; v < W; ++v) total_parked += sh.cnt_parked[v];
        if (total_parked >= 2 && wave == 0) {
#pragma unroll 1
            for (int j = 0; j < W; ++j) {
                const int xx = lane + kWave * j;
                sh.jmp[0][xx] = sh.f[xx];
                sh.mark[xx] = 0;
                sh.ent[xx] = -1;
            }
            wave_lds_sync();
#pragma unroll 1
            for (int d = 0; d < kLogNW; ++d) {
                const int src = d & 1;
#pragma unroll 1
                for (int j = 0; j < W; ++j) {
                    const int xx = lane + kWave * j;
                    sh.jmp[src ^ 1][xx] = sh.jmp[src][sh.jmp[src][xx]];
                }
                wave_lds_sync();
            }
            // jmp[kLogNW & 1][x] = f^NW(x), a node on the cycle x leads into
#pragma unroll 1
            for (int j = 0; j < W; ++j) sh.mark[sh.jmp[kLogNW & 1][lane + kWave * j]] = 1;
            wave_lds_sync();
            bool any = false;
#pragma unroll 1
            for (int j = 0; j < W; ++j) {
                const int xx = lane + kWave * j;
                const int fx = sh.f[xx];
                if (fx != xx && sh.mark[xx]) {
                    sh.ent[fx] = sh.tw[xx];
                    any = true;
                }
            }
            if (__ballot(any) && lane == 0) ++ws.pops;
        }

        // ==== B6
        __syncthreads();

        if (total_parked >= 2 && parked && !bad) {
            const int32_t en = sh.ent[tid];
            if (en >= 0) {
                e = en;
                parked = false;
                if (mem) {
                    mode = (e == h) ? kDraw : kPopLoad;
                } else {
                    int p = -1;
                    for (int j = 0; j < depth; ++j)
                        if (sh.stk_node[j][tid] == e) p = j;
                    if (p < 0) {
                        bad = true;
                        raise_err(c.err, kErrInconsistent, -4);
                        sh.flag[par] = 1;
                    } else {
                        rel_lo = p + 1;
                        rel_hi = depth;
                        depth = p + 1;
                        if (e != h) {
                            h = e;
                            kh = sh.stk_k[p][tid];
                            mode = kNbLoad;
                        } else {
                            mode = kDraw;
                        }
                    }
                }
            }
        }

        // ---- released nodes: free words; those behind the scan go on the revisit list
        auto push_one = [&](int32_t node) {
            const int idx = atomicAdd(&sh.push_cnt[par], 1);
            if (rev_n + idx < kGroupRevCap)
                sh.rev[rev_n + idx] = node;
            else
                sh.ovf[par] = 1;
        };
        if (push && pos_of(pushed) < cursor) push_one(pushed);
        for (int j = rel_lo; j < rel_hi; ++j) {
            const int32_t node = sh.stk_node[j][tid];
            st[node] = st_pack(-1, sh.stk_k[j][tid], kTagFree, ep);
            if (pos_of(node) < cursor) push_one(node);
        }
        fresh = fresh && bad;
        const uint64_t idle_end = __ballot(mode == kIdle);
        const int64_t tsum = wave_sum_i64(tree_local);
        if (lane == 0) {
            sh.cnt_idle[wave] = __popcll(idle_end);
            sh.part[wave] = tsum;
        }
        if (tid == 0) {
            ++ws.iters;
            ws.idle += (unsigned long long)total_idle;
            ws.parked += (unsigned long long)total_parked;
        }
    }
    // leave the sample's stores visible before the slot is reused; sum the draws
    __syncthreads();
    const int64_t ysum = wave_sum_i64(y1_local);
    if (lane == 0) sh.part[wave] = ysum;
    __syncthreads();
    int64_t y = 0;
#pragma unroll
    for (int v = 0; v < W; ++v) y += sh.part[v];
    *y1_out = y;
    __syncthreads();
    return true;
}

// statistics of a workgroup: every wave adds its walkers' draws, thread 0
// the per-round counters it kept
static __device__ void flush_group_stats(const WaveStats &ws, unsigned long long *stats) {
    const int64_t d = wave_sum_i64((int64_t)ws.draws);
    if ((threadIdx.x & (kWave - 1)) == 0) atomicAdd(&stats[kStatDraws], (unsigned long long)d);
    if (threadIdx.x == 0) {
        atomicAdd(&stats[kStatIters], ws.iters);
        atomicAdd(&stats[kStatTrees], ws.trees);
        atomicAdd(&stats[kStatPops], ws.pops);
        atomicAdd(&stats[kStatRescans], ws.rescans);
        atomicAdd(&stats[kStatIdleLanes], ws.idle);
        atomicAdd(&stats[kStatParkedLanes], ws.parked);
    }
}

}  // namespace lap
