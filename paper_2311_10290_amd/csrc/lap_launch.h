// Host-side launchers of the library's kernels (one per kernel family).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "lap_device.h"
#include "lap_params.h"

namespace lap {

hipError_t launch_wilson_lane(const WilsonParams &p, int64_t slots, hipStream_t s);
// lanes: samples per workgroup (one wavefront), with lds_bytes(n, nnz, lanes)
// of LDS; slots: samples run at once (at most 2^16 workgroups), each lane
// taking every slots-th sample; p.state and p.slot_epoch are not used
hipError_t launch_wilson_lds(const WilsonParams &p, int lanes, int64_t slots, hipStream_t s);
hipError_t launch_wilson_wave(const WilsonParams &p, int64_t slots, hipStream_t s);
hipError_t launch_wilson_group(const WilsonParams &p, int64_t slots, int waves, hipStream_t s);
hipError_t launch_absorbed(const AbsorbedParams &p, hipStream_t s);

// Fill n 64-bit words with a value (used instead of hipMemsetAsync so the
// work can sit inside captured graphs).
hipError_t launch_fill_u64(uint64_t *dst, uint64_t value, int64_t n, hipStream_t s);

struct AssembleParams {
    int64_t n;
    int32_t root;
    int32_t n_blocks;
    int64_t omega;                 // samples of the run (sample i -> block floor(i*B/omega))
    const uint64_t *nbr;           // for degrees
    const unsigned long long *y1;  // [B][n]
    const unsigned long long *y2;  // [B][n]
    double *partial;               // [(B+1) * n_parts] scratch
    double *sums;                  // [B+1]: sum_w Y2_b[w]/d_w, index B = all blocks
    double *trace_parts;           // [n_parts] scratch
    double *diag, *diag_se, *lv_diag, *closeness, *trace;   // outputs (device), each may be null
    double *rw_betweenness, *kirchhoff;
    int32_t n_parts;
};

// Y1[b][u] += count[b] for u != root (device array count[B]).
hipError_t launch_add_baseline(unsigned long long *y1, int64_t n, int32_t root, const int64_t *count, int32_t B,
                               hipStream_t s);

hipError_t launch_assemble_diag(const AssembleParams &p, hipStream_t s);

// Kemeny's constant from per-sample Wilson totals and stationary-start walk
// lengths: kappa = (sum y1 - sum len) / omega and its standard error.
hipError_t launch_kemeny(const int64_t *y1, const int64_t *len, int64_t omega, double *kappa,
                         double *se, hipStream_t s);

hipError_t launch_spantree(const SpanParams &p, hipStream_t s);
hipError_t launch_span_assemble(const SpanAsmParams &p, hipStream_t s);
int64_t span_assemble_parts(int64_t n);
hipError_t launch_loop_included(const LoopParams &p, hipStream_t s);
hipError_t launch_pair_paths(const PairParams &p, bool hashed, hipStream_t s);
hipError_t launch_pair_assemble(const PairAsmParams &p, hipStream_t s);
hipError_t launch_lv_rows(const unsigned long long *Y, const uint64_t *nbr, int64_t n, int64_t n_src, int32_t B,
                          int64_t omega, int32_t root, double *out, hipStream_t s);
hipError_t launch_serve(const ServeParams &p, int64_t waves, hipStream_t s);
hipError_t launch_serve_group(const ServeParams &p, int waves, int64_t groups, hipStream_t s);
hipError_t launch_batch(const BatchParams &p, int64_t waves, hipStream_t s);
hipError_t launch_batch_assemble(const BatchParams &p, int32_t n_jobs, hipStream_t s);

}  // namespace lap
