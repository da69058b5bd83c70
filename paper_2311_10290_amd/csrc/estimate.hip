// v-absorbed walks and the FP64 estimator assembly.
//
// absorbed_kernel: one lane per walk (the second phase of Alg. 2 with a
// uniform start over all of V, and the y2 walk of Alg. 4 with a start drawn
// from the stationary distribution).  Every departure from a node counts one
// visit of that node and one unit of length; the arrival at v ends the walk.
//
// Assembly (Alg. 2 last loop, the closeness formula of Sec. 2, Alg. 4 update)
// from exact integer counts in FP64:
//   S_b    = sum_w Y2_b[w] / d_w  per block b,  S = sum_b S_b
//   diag_u = (Y1[u] - 2 Y2[u]) / (omega d_u) + S / (omega n)
//   c_u    = (n-1) / (Tr + n diag_u),  Tr = sum_u diag_u
//   kappa  = (sum_i y1_i - sum_i len_i) / omega
// Standard errors: batch means over the B sample blocks for diag; the sample
// standard deviation of y1_i - len_i over sqrt(omega) for kappa.  Sums run in a
// fixed order (per-thread strides, then a tree), so results are reproducible.
#include "lap_device.h"
#include "lap_launch.h"
#include "walks.h"

namespace lap {

// Both walk kinds in one grid (blockIdx.y picks the kind), so a step waits for
// the longer of the two longest walks, not their sum.  The walks are few
// single-lane chains that overlap the Wilson kernel on the same CUs; they run
// at raised wave priority so each of their dependent steps issues promptly.
__global__ __launch_bounds__(64) void absorbed_kernel(AbsorbedParams p) {
    __builtin_amdgcn_s_setprio(3);
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const uint64_t t0 = wall_clock64();
    const uint32_t tag = (p.kinds == 2 || blockIdx.y == 1) ? 2u : 1u;
    unsigned long long *y2 = tag == 1 ? p.y2 : nullptr;
    int64_t *len_out = tag == 1 ? p.len_u : p.len_p;
    const WalkGraph g{p.nbr, p.col, p.arcs, p.n, p.nnz, p.root, p.k0, p.k1, p.qid};
    unsigned long long steps = 0;
    for (int64_t wi = gid; wi < p.n_walks; wi += stride) {
        const int64_t i = p.walk_begin + wi;
        unsigned long long *y2b = y2 ? y2 + ((i * (int64_t)p.n_blocks) / p.n_total) * p.n : nullptr;
        const int64_t len = absorbed_walk(g, tag, i, y2b, p.err, t0, p.deadline);
        if (len < 0) break;
        if (len_out) len_out[wi] = len;
        steps += (unsigned long long)len;
    }
    atomicAdd(&p.stats[kStatAbsorbed], steps);
}

hipError_t launch_absorbed(const AbsorbedParams &p, hipStream_t s) {
    if (p.kinds < 1 || p.kinds > 3) return hipErrorInvalidValue;
    const int bs = 64;
    int64_t grid = (p.n_walks + bs - 1) / bs;
    if (grid < 1) grid = 1;
    const unsigned n_kinds = p.kinds == 3 ? 2u : 1u;
    hipLaunchKernelGGL(absorbed_kernel, dim3((unsigned)grid, n_kinds), dim3(bs), 0, s, p);
    return hipGetLastError();
}

// 16-byte stores over the 16-byte aligned body; the word before it (when the
// buffer starts 8 bytes past a 16-byte boundary) and the word after it (odd
// length) are stored by the first thread.
typedef unsigned long long u64x2 __attribute__((ext_vector_type(2)));

__global__ void fill_u64_kernel(uint64_t *dst, uint64_t value, int64_t n) {
    const int64_t head = ((uintptr_t)dst & 15) ? 1 : 0;
    const int64_t pairs = (n - head) / 2;
    u64x2 *body = reinterpret_cast<u64x2 *>(dst + head);
    const u64x2 w = {value, value};
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < pairs; i += stride) body[i] = w;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        if (head) dst[0] = value;
        if (head + 2 * pairs < n) dst[n - 1] = value;
    }
}

hipError_t launch_fill_u64(uint64_t *dst, uint64_t value, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t grid = (n / 2 + 255) / 256;
    if (grid < 1) grid = 1;
    if (grid > 65536) grid = 65536;
    hipLaunchKernelGGL(fill_u64_kernel, dim3((unsigned)grid), dim3(256), 0, s, dst, value, n);
    return hipGetLastError();
}

// ----------------------------------------------------------------- reductions
template <int BS>
__device__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
#pragma unroll
    for (int off = BS / 2; off > 0; off >>= 1) {
        if (t < off) sh[t] += sh[t + off];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

constexpr int kAsmBS = 256;

__device__ __forceinline__ double deg_of(const uint64_t *nbr, int64_t u) { return (double)nbr_deg(nbr[u]); }

// partial[b * n_parts + part] = sum over this part's nodes of Y2_b[w] / d_w.
// Workgroups of one part for consecutive blocks are launched together, so the
// part's degrees are read from L2 after the first.
__global__ __launch_bounds__(kAsmBS) void y2_sums_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    const int b = blockIdx.x;
    const int64_t per = (p.n + p.n_parts - 1) / p.n_parts;
    const int64_t lo = (int64_t)blockIdx.y * per, hi = min(p.n, lo + per);
    const unsigned long long *y2 = p.y2 + (int64_t)b * p.n;
    double acc = 0.0;
    for (int64_t w = lo + threadIdx.x; w < hi; w += kAsmBS)
        if (w != p.root) acc += (double)y2[w] / deg_of(p.nbr, w);
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.partial[(int64_t)b * p.n_parts + blockIdx.y] = s;
}

// sums[b] = S_b, one workgroup per block
__global__ __launch_bounds__(kAsmBS) void y2_sums_final_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < p.n_parts; i += kAsmBS) acc += p.partial[(int64_t)b * p.n_parts + i];
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.sums[b] = s;
}

// sums[B] = S = sum_b S_b (every visit belongs to exactly one block)
__global__ __launch_bounds__(kAsmBS) void y2_total_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    double acc = 0.0;
    for (int b = threadIdx.x; b < p.n_blocks; b += kAsmBS) acc += p.sums[b];
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.sums[p.n_blocks] = s;
}

__device__ __forceinline__ int64_t block_count(int64_t omega, int32_t B, int32_t b) {
    // number of i in [0, omega) with floor(i*B/omega) == b
    const int64_t lo = ((int64_t)b * omega + B - 1) / B;
    const int64_t hi = ((int64_t)(b + 1) * omega + B - 1) / B;
    return hi - lo;
}

// Per-block constants of diag_kernel: sample count omega_b, 1/omega_b and
// S_b/(omega_b n), in LDS when there are at most kAsmTab blocks.
constexpr int kAsmTab = 1024;

struct BlockConst {
    unsigned long long cnt;
    double scale, glob;
};

__device__ __forceinline__ BlockConst block_const(const AssembleParams &p, int b, double nn) {
    const int64_t ob = block_count(p.omega, p.n_blocks, b);
    return BlockConst{(unsigned long long)ob, 1.0 / (double)ob, p.sums[b] / ((double)ob * nn)};
}

// diag_u, its batch-means standard error and (L_v^-1)_uu; per-part sums of
// diag_u for the trace.  The spread over blocks is accumulated as sums of
// v_b - v_0 and its square (shifted data), which needs no division per block.
template <bool TAB>
__global__ __launch_bounds__(kAsmBS) void diag_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    __shared__ BlockConst tab[TAB ? kAsmTab : 1];
    const int B = p.n_blocks;
    const double nn = (double)p.n;
    if (TAB) {
        for (int b = threadIdx.x; b < B; b += kAsmBS) tab[b] = block_const(p, b, nn);
        __syncthreads();
    }
    auto bc = [&](int b) -> BlockConst { return TAB ? tab[b] : block_const(p, b, nn); };
    const int64_t per = (p.n + p.n_parts - 1) / p.n_parts;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(p.n, lo + per);
    const double om = (double)p.omega;
    double tr = 0.0;
    for (int64_t u = lo + threadIdx.x; u < hi; u += kAsmBS) {
        double diag, lv = 0.0, k = 0.0, s1 = 0.0, s2 = 0.0;
        if (u == p.root) {
            diag = p.sums[B] / (om * nn);
            for (int b = 0; b < B; ++b) {
                const double v = bc(b).glob;
                if (b == 0) k = v;
                s1 += v - k;
                s2 += (v - k) * (v - k);
            }
        } else {
            const double du = deg_of(p.nbr, u);
            const double inv_du = 1.0 / du;
            unsigned long long a1 = 0, a2 = 0;
#pragma unroll 8
            for (int b = 0; b < B; ++b) {
                const BlockConst c = bc(b);
                // counts hold draws beyond the first; add the one-per-sample baseline
                const unsigned long long c1 = p.y1[(int64_t)b * p.n + u] + c.cnt;
                const unsigned long long c2 = p.y2[(int64_t)b * p.n + u];
                a1 += c1;
                a2 += c2;
                const double v = ((double)c1 - 2.0 * (double)c2) * (c.scale * inv_du) + c.glob;
                if (b == 0) k = v;
                s1 += v - k;
                s2 += (v - k) * (v - k);
            }
            diag = ((double)a1 - 2.0 * (double)a2) / (om * du) + p.sums[B] / (om * nn);
            lv = (double)a1 / (om * du);
        }
        if (p.diag) p.diag[u] = diag;
        if (p.diag_se) {
            double se = __builtin_nan("");
            if (B > 1) se = sqrt(fmax(0.0, (s2 - s1 * s1 / (double)B) / (double)(B - 1)) / (double)B);
            p.diag_se[u] = se;
        }
        if (p.lv_diag) p.lv_diag[u] = lv;
        tr += diag;
    }
    const double s = block_sum<kAsmBS>(tr, sh);
    if (threadIdx.x == 0) p.trace_parts[blockIdx.x] = s;
}

__global__ __launch_bounds__(kAsmBS) void trace_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    double acc = 0.0;
    for (int i = threadIdx.x; i < p.n_parts; i += kAsmBS) acc += p.trace_parts[i];
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.sums[p.n_blocks + 1] = s;
    if (threadIdx.x == 0 && p.trace) p.trace[0] = s;
    if (threadIdx.x == 0 && p.kirchhoff) p.kirchhoff[0] = (double)p.n * s;   // n Tr(L^dagger)
}

// c_u = (n-1)/(Tr + n diag_u) (Sec. 2); random-walk betweenness
// 1/n + Tr/((n-1)(Tr + n diag_u)) (end of Sec. 5)
__global__ __launch_bounds__(kAsmBS) void closeness_kernel(AssembleParams p, const double *diag) {
    const double tr = p.sums[p.n_blocks + 1];
    const double nn = (double)p.n;
    for (int64_t u = (int64_t)blockIdx.x * kAsmBS + threadIdx.x; u < p.n; u += (int64_t)gridDim.x * kAsmBS) {
        const double den = tr + nn * diag[u];
        if (p.closeness) p.closeness[u] = (nn - 1.0) / den;
        if (p.rw_betweenness) p.rw_betweenness[u] = 1.0 / nn + tr / ((nn - 1.0) * den);
    }
}

hipError_t launch_assemble_diag(const AssembleParams &p, hipStream_t s) {
    if (p.n_parts < 1 || p.n_parts > 65535 || p.n_blocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(y2_sums_kernel, dim3((unsigned)p.n_blocks, (unsigned)p.n_parts), dim3(kAsmBS), 0, s, p);
    hipLaunchKernelGGL(y2_sums_final_kernel, dim3((unsigned)p.n_blocks), dim3(kAsmBS), 0, s, p);
    hipLaunchKernelGGL(y2_total_kernel, dim3(1), dim3(kAsmBS), 0, s, p);
    if (p.n_blocks <= kAsmTab)
        hipLaunchKernelGGL(diag_kernel<true>, dim3((unsigned)p.n_parts), dim3(kAsmBS), 0, s, p);
    else
        hipLaunchKernelGGL(diag_kernel<false>, dim3((unsigned)p.n_parts), dim3(kAsmBS), 0, s, p);
    hipLaunchKernelGGL(trace_kernel, dim3(1), dim3(kAsmBS), 0, s, p);
    if (p.closeness || p.rw_betweenness) {
        int64_t grid = (p.n + kAsmBS - 1) / kAsmBS;
        if (grid > 4096) grid = 4096;
        hipLaunchKernelGGL(closeness_kernel, dim3((unsigned)grid), dim3(kAsmBS), 0, s, p, p.diag);
    }
    return hipGetLastError();
}

__global__ __launch_bounds__(kAsmBS) void kemeny_kernel(const int64_t *y1, const int64_t *len, int64_t omega,
                                                      double *kappa, double *se) {
    __shared__ double sh[kAsmBS];
    __shared__ long long shi[kAsmBS];
    const int t = threadIdx.x;
    long long acc = 0;
    for (int64_t i = t; i < omega; i += kAsmBS) acc += (long long)(y1[i] - len[i]);
    shi[t] = acc;
    __syncthreads();
    for (int off = kAsmBS / 2; off > 0; off >>= 1) {
        if (t < off) shi[t] += shi[t + off];
        __syncthreads();
    }
    const long long total = shi[0];
    const double mean = (double)total / (double)omega;
    double sq = 0.0;
    for (int64_t i = t; i < omega; i += kAsmBS) {
        const double d = (double)(y1[i] - len[i]) - mean;
        sq += d * d;
    }
    const double s2 = block_sum<kAsmBS>(sq, sh);
    if (t == 0) {
        if (kappa) kappa[0] = mean;
        if (se) se[0] = (omega > 1) ? sqrt(s2 / (double)(omega - 1)) / sqrt((double)omega) : __builtin_nan("");
    }
}

// Y1[b][u] += count[b] for every u != root: restores full draw counts from
// the kernels' draws-beyond-the-first.
__global__ void add_baseline_kernel(unsigned long long *y1, int64_t n, int32_t root, const int64_t *count, int32_t B) {
    const int64_t total = (int64_t)B * n;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < total; i += stride) {
        const int64_t u = i % n;
        if (u != root) y1[i] += (unsigned long long)count[i / n];
    }
}

hipError_t launch_add_baseline(unsigned long long *y1, int64_t n, int32_t root, const int64_t *count, int32_t B,
                               hipStream_t s) {
    int64_t grid = ((int64_t)B * n + 255) / 256;
    if (grid > 8192) grid = 8192;
    if (grid < 1) grid = 1;
    hipLaunchKernelGGL(add_baseline_kernel, dim3((unsigned)grid), dim3(256), 0, s, y1, n, root, count, B);
    return hipGetLastError();
}

hipError_t launch_kemeny(const int64_t *y1, const int64_t *len, int64_t omega, double *kappa, double *se,
                         hipStream_t s) {
    hipLaunchKernelGGL(kemeny_kernel, dim3(1), dim3(kAsmBS), 0, s, y1, len, omega, kappa, se);
    return hipGetLastError();
}

}  // namespace lap
