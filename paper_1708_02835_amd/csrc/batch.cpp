// One step of many independent tiled factorisations in fused launches (see
// batch.hpp): fills the prefix offsets of the descriptors, copies them to the
// device and enqueues the launches.
#include "batch.hpp"

namespace gl {

int enqueue_step(BatchReq *d, BatchReq *dev, int count, int b, hipStream_t s, int *launches)
{
    int64_t o_stage = 0, o_gen = 0, o_trsm = 0, o_tr = 0;
    const int64_t sub = (int64_t)(b / 128) * (b / 128);
    bool any_new = false, any_fin = false, euclid = true;
    for (int i = 0; i < count; ++i) {
        BatchReq &q = d[i];
        q.o_stage = o_stage;
        q.o_gen = o_gen;
        q.o_trsm = o_trsm;
        q.o_tr = o_tr;
        if (q.is_new) {
            o_stage += ceil_div(q.npad, 256);
            o_gen += tile_count(q.nt);
            any_new = true;
            euclid = euclid && q.geo.metric == GL_EUCLIDEAN;
        }
        const int64_t m = q.nt - q.k - 1;
        o_trsm += m * (b / 64);
        o_tr += m * (m + 1) / 2 * sub;
        any_fin = any_fin || q.finishing;
    }
    GL_HIP_TRY(hipMemcpyAsync(dev, d, count * sizeof(BatchReq), hipMemcpyHostToDevice, s));
    int n = 0;
    if (any_new) {
        launch_stage_batched(dev, count, o_stage, s);
        launch_gen_batched(b, dev, count, o_gen, euclid, s);
        n += 2;
    }
    launch_potrf_batched(b, dev, count, s);
    launch_fwd_diag_batched(b, dev, count, s);
    launch_trsm_batched(b, dev, count, o_trsm, s);
    launch_fwd_update_batched(b, dev, count, o_trsm, s);
    launch_trailing_batched(b, dev, count, o_tr, s);
    n += 5;
    if (any_fin) {
        launch_final_batched(dev, count, s);
        ++n;
    }
    GL_HIP_TRY(hipGetLastError());
    if (launches) *launches = n;
    return GL_OK;
}

}  // namespace gl
