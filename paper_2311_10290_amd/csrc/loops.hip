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

}  // namespace lap
