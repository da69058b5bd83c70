// v-absorbed walks and the FP64 estimator assembly.
//
// absorbed_kernel: one lane per walk (the second phase of Alg. 2 with a
// uniform start over all of V, and the y2 walk of Alg. 4 with a start drawn
// from the stationary distribution).  Every departure from a node counts one
// visit of that node and one unit of length; the arrival at v ends the walk.
//
// Assembly (Alg. 2 last loop, the closeness formula of Sec. 2, Alg. 4 update)
// from exact integer counts, dividing once in FP64:
//   S_b    = sum_w Y2_b[w] / d_w                         per block b and overall
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

__global__ void fill_u64_kernel(uint64_t *dst, uint64_t value, int64_t n) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) dst[i] = value;
}

hipError_t launch_fill_u64(uint64_t *dst, uint64_t value, int64_t n, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t grid = (n + 255) / 256;
    if (grid > 4096) grid = 4096;
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

// partial[b * n_parts + part] = sum over this part's nodes of Y2_b[w] / d_w
// (b == B: all blocks together)
__global__ __launch_bounds__(kAsmBS) void y2_sums_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    const int b = blockIdx.y;
    const int64_t per = (p.n + p.n_parts - 1) / p.n_parts;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(p.n, lo + per);
    double acc = 0.0;
    for (int64_t w = lo + threadIdx.x; w < hi; w += kAsmBS) {
        if (w == p.root) continue;
        unsigned long long c;
        if (b < p.n_blocks) {
            c = p.y2[(int64_t)b * p.n + w];
        } else {
            c = 0;
            for (int q = 0; q < p.n_blocks; ++q) c += p.y2[(int64_t)q * p.n + w];
        }
        acc += (double)c / deg_of(p.nbr, w);
    }
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.partial[(int64_t)b * p.n_parts + blockIdx.x] = s;
}

__global__ __launch_bounds__(kAsmBS) void y2_sums_final_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    const int b = blockIdx.x;
    double acc = 0.0;
    for (int i = threadIdx.x; i < p.n_parts; i += kAsmBS) acc += p.partial[(int64_t)b * p.n_parts + i];
    const double s = block_sum<kAsmBS>(acc, sh);
    if (threadIdx.x == 0) p.sums[b] = s;
}

__device__ __forceinline__ int64_t block_count(int64_t omega, int32_t B, int32_t b) {
    // number of i in [0, omega) with floor(i*B/omega) == b
    const int64_t lo = ((int64_t)b * omega + B - 1) / B;
    const int64_t hi = ((int64_t)(b + 1) * omega + B - 1) / B;
    return hi - lo;
}

__global__ __launch_bounds__(kAsmBS) void diag_kernel(AssembleParams p) {
    __shared__ double sh[kAsmBS];
    const int64_t per = (p.n + p.n_parts - 1) / p.n_parts;
    const int64_t lo = (int64_t)blockIdx.x * per, hi = min(p.n, lo + per);
    const double nn = (double)p.n;
    double tr = 0.0;
    for (int64_t u = lo + threadIdx.x; u < hi; u += kAsmBS) {
        double diag, se = 0.0, lv = 0.0;
        if (u == p.root) {
            diag = p.sums[p.n_blocks] / ((double)p.omega * nn);
            if (p.n_blocks > 1) {
                double m = 0.0, m2 = 0.0;
                for (int b = 0; b < p.n_blocks; ++b) {
                    const double ob = (double)block_count(p.omega, p.n_blocks, b);
                    const double v = p.sums[b] / (ob * nn);
                    const double d = v - m;
                    m += d / (b + 1);
                    m2 += d * (v - m);
                }
                se = sqrt(m2 / (p.n_blocks - 1)) / sqrt((double)p.n_blocks);
            }
        } else {
            const double du = deg_of(p.nbr, u);
            unsigned long long a1 = 0, a2 = 0;
            double m = 0.0, m2 = 0.0;
            for (int b = 0; b < p.n_blocks; ++b) {
                // counts hold draws beyond the first; add the one-per-sample baseline
                const unsigned long long c1 =
                    p.y1[(int64_t)b * p.n + u] + (unsigned long long)block_count(p.omega, p.n_blocks, b);
                const unsigned long long c2 = p.y2[(int64_t)b * p.n + u];
                a1 += c1;
                a2 += c2;
                if (p.n_blocks > 1) {
                    const double ob = (double)block_count(p.omega, p.n_blocks, b);
                    const double v = ((double)c1 - 2.0 * (double)c2) / (ob * du) + p.sums[b] / (ob * nn);
                    const double d = v - m;
                    m += d / (b + 1);
                    m2 += d * (v - m);
                }
            }
            const double om = (double)p.omega;
            diag = ((double)a1 - 2.0 * (double)a2) / (om * du) + p.sums[p.n_blocks] / (om * nn);
            lv = (double)a1 / (om * du);
            if (p.n_blocks > 1) se = sqrt(m2 / (p.n_blocks - 1)) / sqrt((double)p.n_blocks);
        }
        if (p.diag) p.diag[u] = diag;
        if (p.diag_se) p.diag_se[u] = (p.n_blocks > 1) ? se : __builtin_nan("");
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
    hipLaunchKernelGGL(y2_sums_kernel, dim3((unsigned)p.n_parts, (unsigned)(p.n_blocks + 1)), dim3(kAsmBS),
                       0, s, p);
    hipLaunchKernelGGL(y2_sums_final_kernel, dim3((unsigned)(p.n_blocks + 1)), dim3(kAsmBS), 0, s, p);
    hipLaunchKernelGGL(diag_kernel, dim3((unsigned)p.n_parts), dim3(kAsmBS), 0, s, p);
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
