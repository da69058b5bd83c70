// SpanTree estimators (Alg. 1 for diag(L^dagger) and closeness, Alg. 3 for
// Kemeny's constant) on the spanning trees the Wilson kernels leave in their
// state slots: after a launch with at most one sample per slot, slot s holds
// sample s's tree as the next fields of its state words.
//
// One workgroup processes one tree (n nodes) in six steps over the slot's
// scratch arrays, with a barrier between steps:
//   1. child counts;
//   2. subtree sizes sz and degree sums psd, bottom-up: every leaf climbs
//      towards v, and at each parent the last child to arrive carries the
//      climb on (so every node is finished exactly once).  A child adds its
//      size and takes one off the parent's child count in one atomic on a
//      packed (count, size) word, so the last child reads the parent's final
//      size from that atomic's return value;
//   3. sibling offsets: each child reserves a range of its parent's
//      subtree (any order of siblings gives a valid pre-order);
//   4. pre-order numbers by pointer jumping on packed (sum, pointer) words,
//      in place: pre[u] = sum over u's tree path (without v) of 1 + offset,
//      so u's subtree is [pre[u], pre[u] + sz[u]).  A word is read and
//      written whole, so a node reads either the old or the new (sum,
//      pointer) pair of the node it jumps over, and either keeps the sum
//      equal to the weights from u up to (not including) the pointer;
//   5. the BFS-path pass: for every u, each edge (e1, e2) of u's BFS path
//      that is a tree edge on u's tree path adds its flow in the direction
//      e1 -> e2: +1 / -1 to x1(u), +/- the path support (sz for unit weights,
//      psd for degree weights) to x2(u) (Alg. 1 and Alg. 3, inner loops);
//   6. the sample's sums: x1(u), x2(u) (sz) are added to the per-node block
//      counts, sum_u d_u x1(u) and sum_u d_u x2(u) (psd) to the per-sample
//      Kemeny terms.
// Path support is kept in integer units (1/n for Alg. 1, 1/2m for Alg. 3),
// so every output is an exact integer and independent of thread timing.
#include "lap_device.h"
#include "lap_launch.h"

namespace lap {

constexpr int kSpanThreads = 256;
constexpr int kSpanWave = 64;
constexpr int kJumpBatch = 8;   // nodes whose jumps one thread has in flight

struct SpanScratch {
    int64_t *psd;    // degree sums of subtrees
    uint64_t *cs;    // child count << 32 | subtree size
    uint64_t *su;    // pre-order partial sum << 32 | jump pointer
    int32_t *acc, *off, *leaf;
};

__device__ __forceinline__ SpanScratch span_scratch(const SpanParams &p, int64_t slot) {
    SpanScratch s;
    int64_t *a = p.scratch64 + slot * kSpanInt64PerNode * p.n;
    s.psd = a;
    s.cs = (uint64_t *)(a + p.n);
    s.su = (uint64_t *)(a + 2 * p.n);
    int32_t *b = p.scratch32 + slot * kSpanInt32PerNode * p.n;
    s.acc = b;
    s.off = b + p.n;
    s.leaf = b + 2 * p.n;
    return s;
}

__device__ __forceinline__ int64_t span_block(int64_t sample, int32_t B, int64_t n_total) {
    return (sample * (int64_t)B) / n_total;
}

__device__ __forceinline__ int32_t cs_size(uint64_t w) { return (int32_t)(uint32_t)w; }
__device__ __forceinline__ int32_t su_sum(uint64_t w) { return (int32_t)(uint32_t)(w >> 32); }
__device__ __forceinline__ int32_t su_ptr(uint64_t w) { return (int32_t)(uint32_t)w; }
__device__ __forceinline__ uint64_t su_pack(int32_t sum, int32_t ptr) {
    return ((uint64_t)(uint32_t)sum << 32) | (uint64_t)(uint32_t)ptr;
}

// A tree is processed by one workgroup only, so every exchange below is
// between threads of one workgroup (one CU): workgroup-scope atomics and
// fences suffice and keep the L2 out of it.
template <class T>
__device__ __forceinline__ T ld_wg(const T *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
template <class T>
__device__ __forceinline__ void st_wg(T *p, T v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void add_wg(int64_t *p, int64_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void add_wg(uint64_t *p, uint64_t v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// all threads of the workgroup: barrier with workgroup-scope release/acquire
__device__ __forceinline__ void span_sync() { __syncthreads(); }

__global__ __launch_bounds__(kSpanThreads) void spantree_kernel(SpanParams p) {
    __shared__ int32_t flag, bad;
    __shared__ long long red1[kSpanThreads / kSpanWave], red2[kSpanThreads / kSpanWave];
    const int tid = (int)threadIdx.x;
    const int64_t slot = blockIdx.x;
    if (slot >= p.n_trees) return;
    const int64_t n = p.n;
    const int32_t root = p.root;
    const uint64_t *st = p.state + slot * n;
    SpanScratch s = span_scratch(p, slot);
    const int64_t sample = p.sample_begin + slot;

    // 1. initial values (no children, size 1, own degree) and child counts;
    // every parent must be a node
    if (tid == 0) bad = 0;
    for (int64_t a = tid; a < n; a += kSpanThreads) {
        s.cs[a] = 1ull;
        s.psd[a] = (int64_t)nbr_deg(p.nbr[a]);
        s.acc[a] = 0;
    }
    span_sync();
    for (int64_t u = tid; u < n; u += kSpanThreads)
        if (u != root) {
            const int32_t nx = st_next(st[u]);
            if (nx < 0 || nx >= n || nx == u) {
                raise_err(p.err, kErrInconsistent, -10);
                bad = 1;
            } else {
                add_wg(&s.cs[nx], 1ull << 32);
            }
        }
    span_sync();
    if (bad) return;   // the same LDS value for every thread after the barrier
    // the leaves, fixed before any count is consumed
    for (int64_t u = tid; u < n; u += kSpanThreads) s.leaf[u] = (int32_t)(ld_wg(&s.cs[u]) >> 32);
    span_sync();

    // 2. bottom-up sums: leaves climb; the last child at a parent continues
    // with the parent's final size (from its atomic) and degree sum
    for (int64_t u = tid; u < n; u += kSpanThreads) {
        if (u == root || s.leaf[u] != 0) continue;
        int32_t za = 1;
        int64_t pa = (int64_t)nbr_deg(p.nbr[u]);
        int32_t par = st_next(st[u]);
        for (int64_t guard = 0; guard < n; ++guard) {
            add_wg(&s.psd[par], pa);
            // size += za and count -= 1 in one word; release: the degree sum
            // above is visible to whichever child arrives last
            const uint64_t old = __hip_atomic_fetch_add(&s.cs[par], (uint64_t)(uint32_t)za - (1ull << 32),
                                                        __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_WORKGROUP);
            if ((old >> 32) != 1ull || par == root) break;
            za += cs_size(old);
            const int32_t a = par;
            pa = ld_wg(&s.psd[a]);
            par = st_next(st[a]);
        }
    }
    span_sync();

    // 3. sibling offsets
    for (int64_t u = tid; u < n; u += kSpanThreads)
        if (u != root)
            s.off[u] = __hip_atomic_fetch_add(&s.acc[st_next(st[u])], cs_size(ld_wg(&s.cs[u])), __ATOMIC_RELAXED,
                                              __HIP_MEMORY_SCOPE_WORKGROUP);
    span_sync();

    // 4. pre-order numbers: sum = 1 + offset, pointer = parent (v: 0 and v),
    // jumped in place until every pointer is v; the sum is then pre[u]
    for (int64_t u = tid; u < n; u += kSpanThreads)
        st_wg(&s.su[u], (u == root) ? su_pack(0, root) : su_pack(1 + s.off[u], st_next(st[u])));
    for (int round = 0; round < 40; ++round) {
        if (tid == 0) flag = 0;
        __syncthreads();
        bool more = false;
        for (int64_t base = tid; base < n; base += (int64_t)kSpanThreads * kJumpBatch) {
            uint64_t mine[kJumpBatch], up[kJumpBatch];
#pragma unroll
            for (int q = 0; q < kJumpBatch; ++q) {
                const int64_t u = base + (int64_t)q * kSpanThreads;
                mine[q] = (u < n) ? ld_wg(&s.su[u]) : su_pack(0, root);
            }
#pragma unroll
            for (int q = 0; q < kJumpBatch; ++q)
                up[q] = (su_ptr(mine[q]) != root) ? ld_wg(&s.su[su_ptr(mine[q])]) : 0ull;
#pragma unroll
            for (int q = 0; q < kJumpBatch; ++q) {
                const int64_t u = base + (int64_t)q * kSpanThreads;
                if (u < n && su_ptr(mine[q]) != root) {
                    const int32_t next = su_ptr(up[q]);
                    st_wg(&s.su[u], su_pack(su_sum(mine[q]) + su_sum(up[q]), next));
                    more |= (next != root);
                }
            }
        }
        if (more) flag = 1;
        __syncthreads();
        const int f = flag;
        __syncthreads();
        if (!f) break;
    }

    // 5. BFS-path pass, 6. sums
    const int32_t *bp = p.bfs_par;
    unsigned long long *X1 = p.X1 ? p.X1 + span_block(sample, p.n_blocks, p.n_total) * n : nullptr;
    unsigned long long *X2 = p.X2 ? p.X2 + span_block(sample, p.n_blocks, p.n_total) * n : nullptr;
    long long k1 = 0, k2 = 0;
    for (int64_t u = tid; u < n; u += kSpanThreads) {
        const int32_t pu = su_sum(s.su[u]);
        int64_t x1 = 0, x2 = 0, x2d = 0;
        int32_t e1 = (int32_t)u;
        for (int hop = 0; hop < n && e1 != root; ++hop) {
            const int32_t e2 = bp[e1];
            if (st_next(st[e1]) == e2) {
                const int32_t lo = su_sum(s.su[e1]), sz = cs_size(s.cs[e1]);
                if (lo <= pu && pu < lo + sz) {
                    x1 += 1;
                    x2 += sz;
                    x2d += s.psd[e1];
                }
            }
            if (e2 != root && st_next(st[e2]) == e1) {
                const int32_t lo = su_sum(s.su[e2]), sz = cs_size(s.cs[e2]);
                if (lo <= pu && pu < lo + sz) {
                    x1 -= 1;
                    x2 -= sz;
                    x2d -= s.psd[e2];
                }
            }
            e1 = e2;
        }
        if (X1 && x1) atomicAdd(&X1[u], (unsigned long long)x1);
        if (X2 && x2) atomicAdd(&X2[u], (unsigned long long)x2);
        const int64_t d = (int64_t)nbr_deg(p.nbr[u]);
        k1 += d * x1;
        k2 += d * x2d;
    }
    // workgroup sums of the Kemeny terms
#pragma unroll
    for (int off = kSpanWave / 2; off > 0; off >>= 1) {
        k1 += __shfl_xor(k1, off, kSpanWave);
        k2 += __shfl_xor(k2, off, kSpanWave);
    }
    if ((tid & (kSpanWave - 1)) == 0) {
        red1[tid / kSpanWave] = k1;
        red2[tid / kSpanWave] = k2;
    }
    __syncthreads();
    if (tid == 0) {
        long long a = 0, b = 0;
        for (int w = 0; w < kSpanThreads / kSpanWave; ++w) {
            a += red1[w];
            b += red2[w];
        }
        if (p.s1) p.s1[slot] = a;
        if (p.s2) p.s2[slot] = b;
    }
}

// ------------------------------------------------------------------ assembly
// Alg. 1's last loop per block b of omega_b samples: est_b(u) = X1_b(u)/omega_b
// - 2 X2_b(u)/(n omega_b) + sum_w X2_b(w)/(n^2 omega_b); the estimate uses the
// sums over all blocks, the standard error the spread of the block estimates.
// Closeness is (n-1)/(Tr + n diag(u)).  Alg. 3: kappa = mean over samples of
// s1 - s2/2m.  Three launches with fixed-order reductions: block sums of X2
// (exact integers), per-node estimates with per-workgroup partial traces,
// then the trace, closeness and Kemeny's constant.
constexpr int kAsmThreads = 256;

template <class T>
__device__ T asm_reduce(T v, T *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int off = kAsmThreads / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const T r = sh[0];
    __syncthreads();
    return r;
}

// grid = B: blk_sum[b] = sum_u X2_b(u)
__global__ __launch_bounds__(kAsmThreads) void span_blksum_kernel(SpanAsmParams p) {
    __shared__ long long sh[kAsmThreads];
    const int64_t b = blockIdx.x;
    const long long *X2 = (const long long *)p.X2 + b * p.n;
    long long acc = 0;
    for (int64_t u = threadIdx.x; u < p.n; u += kAsmThreads) acc += X2[u];
    const long long r = asm_reduce(acc, sh);
    if (threadIdx.x == 0) p.blk_sum[b] = r;
}

// grid over nodes: diag, diag_se; part[blockIdx] = this workgroup's sum of diag
__global__ __launch_bounds__(kAsmThreads) void span_diag_kernel(SpanAsmParams p) {
    __shared__ double sh[kAsmThreads];
    const int64_t n = p.n;
    const double nn = (double)n, om = (double)p.omega;
    const long long *X1 = (const long long *)p.X1, *X2 = (const long long *)p.X2;
    long long tot = 0;
    for (int32_t b = 0; b < p.B; ++b) tot += p.blk_sum[b];
    const int64_t u = (int64_t)blockIdx.x * kAsmThreads + threadIdx.x;
    double d = 0.0;
    if (u < n) {
        long long x1 = 0, x2 = 0;
        double bs = 0.0;
        auto block_est = [&](int32_t b) {
            const double ob = (double)p.blk_n[b];
            return (double)X1[(int64_t)b * n + u] / ob - 2.0 * (double)X2[(int64_t)b * n + u] / (nn * ob) +
                   (double)p.blk_sum[b] / (nn * nn * ob);
        };
        for (int32_t b = 0; b < p.B; ++b) {
            x1 += X1[(int64_t)b * n + u];
            x2 += X2[(int64_t)b * n + u];
            bs += block_est(b);
        }
        d = (double)x1 / om - 2.0 * (double)x2 / (nn * om) + (double)tot / (nn * nn * om);
        p.diag[u] = d;
        if (p.diag_se) {
            const double B = (double)p.B, mean = bs / B;
            double q = 0.0;
            for (int32_t b = 0; b < p.B; ++b) {
                const double e = block_est(b) - mean;
                q += e * e;
            }
            p.diag_se[u] = p.B > 1 ? sqrt(q / (B - 1.0)) / sqrt(B) : __builtin_nan("");
        }
    }
    const double r = asm_reduce(d, sh);
    if (threadIdx.x == 0) p.part[blockIdx.x] = r;
}

// one workgroup: Tr from the partial sums (fixed order), Kemeny's constant
__global__ __launch_bounds__(kAsmThreads) void span_final_kernel(SpanAsmParams p) {
    __shared__ double sh[kAsmThreads];
    const int t = threadIdx.x;
    if (p.diag) {
        double acc = 0.0;
        for (int64_t i = t; i < p.n_parts; i += kAsmThreads) acc += p.part[i];
        const double Tr = asm_reduce(acc, sh);
        if (t == 0) *p.trace = Tr;
    }
    if (p.kemeny) {
        const double two_m = (double)p.two_m;
        double acc = 0.0;
        for (int64_t i = t; i < p.omega; i += kAsmThreads) acc += (double)p.s1[i] - (double)p.s2[i] / two_m;
        const double mean = asm_reduce(acc, sh) / (double)p.omega;
        double sq = 0.0;
        for (int64_t i = t; i < p.omega; i += kAsmThreads) {
            const double z = (double)p.s1[i] - (double)p.s2[i] / two_m - mean;
            sq += z * z;
        }
        const double SQ = asm_reduce(sq, sh);
        if (t == 0) {
            *p.kemeny = p.n > 1 ? mean : 0.0;
            if (p.kemeny_se)
                *p.kemeny_se = p.omega > 1 ? sqrt(SQ / ((double)p.omega - 1.0)) / sqrt((double)p.omega)
                                           : __builtin_nan("");
        }
    }
}

// grid over nodes: closeness from the trace
__global__ __launch_bounds__(kAsmThreads) void span_closeness_kernel(SpanAsmParams p) {
    const int64_t u = (int64_t)blockIdx.x * kAsmThreads + threadIdx.x;
    const double nn = (double)p.n;
    if (u < p.n) p.closeness[u] = p.n > 1 ? (nn - 1.0) / (*p.trace + nn * p.diag[u]) : 0.0;
}

int64_t span_assemble_parts(int64_t n) { return (n + kAsmThreads - 1) / kAsmThreads; }

hipError_t launch_span_assemble(const SpanAsmParams &p, hipStream_t s) {
    const unsigned g = (unsigned)span_assemble_parts(p.n);
    if (p.diag) {
        hipLaunchKernelGGL(span_blksum_kernel, dim3((unsigned)p.B), dim3(kAsmThreads), 0, s, p);
        hipLaunchKernelGGL(span_diag_kernel, dim3(g), dim3(kAsmThreads), 0, s, p);
    }
    hipLaunchKernelGGL(span_final_kernel, dim3(1), dim3(kAsmThreads), 0, s, p);
    if (p.diag && p.closeness) hipLaunchKernelGGL(span_closeness_kernel, dim3(g), dim3(kAsmThreads), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_spantree(const SpanParams &p, hipStream_t s) {
    hipLaunchKernelGGL(spantree_kernel, dim3((unsigned)p.n_trees), dim3(kSpanThreads), 0, s, p);
    return hipGetLastError();
}

}  // namespace lap
