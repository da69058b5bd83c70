// One v-absorbed walk (the second phase of Alg. 2 for a uniform start, the
// y2 walk of Alg. 4 for a stationary start), shared by the plain and the
// batched kernels.  Every departure from a node counts one visit and one unit
// of length; the arrival at v ends the walk.
#pragma once

#include "lap_device.h"

namespace lap {

// arcs[j] = {target w of CSR slot j, w's adjacency record}: a walk step reads
// its next node and that node's row in one dependent load.  Built only for
// graphs whose column array is too large for the caches (null otherwise: a
// step then reads the target from col and its row from nbr).
struct WalkGraph {
    const uint64_t *nbr;
    const int32_t *col;
    const ulonglong2 *arcs;
    int64_t n, nnz;
    int32_t root;
    uint64_t k0, k1, qid;
};

// Returns the walk's length, or -1 if the time limit passed (p.err is set).
static inline __device__ int64_t absorbed_walk(const WalkGraph &g, uint32_t tag, int64_t i, unsigned long long *y2,
                                        DevErr *err, uint64_t t0, uint64_t deadline) {
    const uint64_t c0 = (uint64_t)i | ((uint64_t)tag << 56);
    const uint64_t x0 = philox_w0(c0, 0, 0, g.qid, g.k0, g.k1);
    // a graph without edges is the single node v: the walk starts (and ends) there
    int32_t u = (tag == 1)      ? (int32_t)pick_below(x0, (uint64_t)g.n)
                : (g.nnz > 0)   ? g.col[pick_below(x0, (uint64_t)g.nnz)]
                                : g.root;
    int64_t len = 0;
    if (g.arcs) {
        // one dependent load per step: the arc gives the next node and its row
        uint64_t nb = (u != g.root) ? g.nbr[u] : 0ull;
        while (u != g.root) {
            if (y2) atomicAdd(&y2[u], 1ull);
            ++len;
            const uint64_t x = philox_w0(c0, (uint64_t)len, 0, g.qid, g.k0, g.k1);
            const ulonglong2 a = g.arcs[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
            u = (int32_t)a.x;
            nb = a.y;
            if ((len & 1023) == 0 && (wall_clock64() - t0 > deadline || err_set(err))) {
                raise_err(err, kErrTimeout, 1);
                return -1;
            }
        }
        return len;
    }
    while (u != g.root) {
        const uint64_t nb = g.nbr[u];
        if (y2) atomicAdd(&y2[u], 1ull);
        ++len;
        const uint64_t x = philox_w0(c0, (uint64_t)len, 0, g.qid, g.k0, g.k1);
        u = g.col[nbr_off(nb) + (int64_t)pick_below(x, nbr_deg(nb))];
        if ((len & 1023) == 0 && (wall_clock64() - t0 > deadline || err_set(err))) {
            raise_err(err, kErrTimeout, 1);
            return -1;
        }
    }
    return len;
}

}  // namespace lap

namespace lap {

// One query walk (Lemma 1; the normalised-length lemma of Sec. 4.3): from a
// given start to the root, the j-th move using counter (i | 3<<56, j, sub,
// qid).  Counts departures from a and from b and sums 1/d over departures in
// walk order.  Returns false if the time limit passed (err is set).
static inline __device__ bool query_walk(const WalkGraph &g, int32_t start, uint32_t sub, int64_t i, int32_t a, int32_t b,
                                  int64_t *dep_a, int64_t *dep_b, double *norm_len, DevErr *err, uint64_t t0,
                                  uint64_t deadline) {
    const uint64_t c0 = (uint64_t)i | (3ull << 56);
    int32_t u = start;
    int64_t da = 0, db = 0, steps = 0;
    double nl = 0.0;
    uint64_t nb = (g.arcs && u != g.root) ? g.nbr[u] : 0ull;
    while (u != g.root) {
        if (!g.arcs) nb = g.nbr[u];
        const uint32_t d = nbr_deg(nb);
        da += (u == a);
        db += (u == b);
        nl += 1.0 / (double)d;
        ++steps;
        const uint64_t x = philox_w0(c0, (uint64_t)steps, sub, g.qid, g.k0, g.k1);
        const int64_t j = nbr_off(nb) + (int64_t)pick_below(x, d);
        if (g.arcs) {
            // one dependent load per step: the arc gives the next node and its row
            const ulonglong2 r = g.arcs[j];
            u = (int32_t)r.x;
            nb = r.y;
        } else {
            u = g.col[j];
        }
        if ((steps & 1023) == 0 && (wall_clock64() - t0 > deadline || err_set(err))) {
            raise_err(err, kErrTimeout, 2);
            return false;
        }
    }
    *dep_a = da;
    *dep_b = db;
    *norm_len = nl;
    return true;
}

}  // namespace lap
