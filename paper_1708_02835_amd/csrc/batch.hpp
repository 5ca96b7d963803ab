// Descriptors of the fused multi-request launches used by the serving loop.
// One launch covers the same step of many resident requests; each request's
// work is a contiguous range of the launch's workgroups, given by exclusive
// prefix offsets, and runs the same per-request code as a single evaluation,
// so a request's arithmetic does not depend on what else is in the launch.
#pragma once

#include "common.hpp"

namespace gl {

struct BatchReq {
    double *tiles, *x, *y, *v, *dinv, *logsum, *quad;
    int64_t *info;
    DevResult *res;
    const double *sx, *sy, *sz;  // dataset (sources of the staging copy)
    gl_theta th;
    Geom geo;
    int64_t n, nt, npad, k;      // k: the step this launch performs
    int64_t o_stage, o_gen, o_trsm, o_tr;
    int32_t is_new, finishing;
};

// Largest request index r with offset(r) <= g (ranges may be empty).
#define GL_BATCH_FIND(d, count, g, field)                    \
    ([&]() {                                                 \
        int r_ = 0;                                          \
        for (int q_ = 1; q_ < (count); ++q_)                 \
            if ((d)[q_].field <= (g)) r_ = q_;               \
        return r_;                                           \
    }())

// Launchers (b = 128, 256, 384, 512); grids come from the totals of the prefix
// offsets.
void launch_stage_batched(const BatchReq *d, int count, int64_t blocks, hipStream_t s);
// euclid: every request that generates in this launch uses the Euclidean distance.
void launch_gen_batched(int b, const BatchReq *d, int count, int64_t tiles, bool euclid, hipStream_t s);
void launch_potrf_batched(int b, const BatchReq *d, int count, hipStream_t s);
void launch_fwd_diag_batched(int b, const BatchReq *d, int count, hipStream_t s);
void launch_trsm_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s);
void launch_fwd_update_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s);
void launch_trailing_batched(int b, const BatchReq *d, int count, int64_t blocks, hipStream_t s);
void launch_final_batched(const BatchReq *d, int count, hipStream_t s);

// One step for d[0..count): the caller sets every field but the offsets
// (k, is_new and finishing included); the offsets are filled in, the array is
// copied to dev (device, count entries) on s and the fused launches follow.
// d must stay valid until the copy has been consumed (pinned memory: until
// the stream passes it).
int enqueue_step(BatchReq *d, BatchReq *dev, int count, int b, hipStream_t s, int *launches);

}  // namespace gl
