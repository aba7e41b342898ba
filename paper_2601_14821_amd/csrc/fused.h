// One view's inputs and outputs for the fused render + removal pass.
#pragma once

#include "common.h"

namespace potr {

struct ViewJob {
    const potr_proj* proj;    // records of this view (N of them)
    const uint32_t* ids;      // sorted splat ids of the call (tile ranges index into it)
    const int32_t* ranges;    // [tiles * 2] half-open ranges of this view
    int32_t W, H, tiles_x, tiles;
    float* image;             // [H*W*3] or null
    const float* target;      // [H*W*3], needed with scores_se
    float* scores;            // [N] += sum |PD|_1, or null (int64 fixed point in that mode)
    float* importance;        // [N] += sum T alpha, or null (likewise)
    float* scores_se;         // [N] += sum dSE, or null (likewise)
    float w_l1, w_im, w_se;   // factors applied to each (tile, splat) partial sum before it is added
};

struct ViewJobs {
    ViewJob j[kViewsPerLaunch];
};

// An output description for N splats x V views: each stride 0 or at least N
// (views must not overlap), each weight finite and > 0, dSE only with a target.
inline potr_status check_outputs(const potr_outputs& o, int64_t N, int32_t V, const float* target) {
    const float* const w[3] = {&o.scores_weight, &o.se_weight, &o.importance_weight};
    const int64_t st[3] = {o.scores_stride, o.se_stride, o.importance_stride};
    const void* const p[3] = {o.scores, o.scores_se, o.importance};
    for (int k = 0; k < 3; ++k) {
        if (!p[k]) continue;
        if (!(*w[k] > 0.f) || *w[k] > 3.0e38f) return fail(POTR_EINVAL, "output %d: weight %g", k, (double)*w[k]);
        if (st[k] < 0 || (st[k] > 0 && st[k] < N) || (st[k] > 0 && V > 1 && st[k] > (int64_t(1) << 40)))
            return fail(POTR_EINVAL, "output %d: stride %lld for N = %lld", k, (long long)st[k], (long long)N);
    }
    if (o.scores_se && !target) return fail(POTR_EINVAL, "scores_se needs a target image");
    if (o.fixed_point != 0 && o.fixed_point != 1) return fail(POTR_EINVAL, "fixed_point %d", o.fixed_point);
    return POTR_OK;
}

// View v's output pointers and weights (no outputs when the scene is empty);
// in fixed point the arrays hold int64 elements.
inline float* view_output(float* base, int64_t stride, int64_t v, bool fixed) {
    if (!base) return nullptr;
    return fixed ? reinterpret_cast<float*>(reinterpret_cast<int64_t*>(base) + v * stride) : base + v * stride;
}
inline void set_outputs(ViewJob& j, const potr_outputs& o, int64_t N, int64_t v) {
    const bool fx = o.fixed_point != 0;
    j.scores = N > 0 ? view_output(o.scores, o.scores_stride, v, fx) : nullptr;
    j.scores_se = N > 0 ? view_output(o.scores_se, o.se_stride, v, fx) : nullptr;
    j.importance = N > 0 ? view_output(o.importance, o.importance_stride, v, fx) : nullptr;
    j.w_l1 = o.scores_weight;
    j.w_se = o.se_weight;
    j.w_im = o.importance_weight;
}

// dynamic LDS bytes of the fused pass with n_out per-splat outputs (fx: in
// fixed point, 8-byte per-entry sums)
size_t fused_smem_bytes(const potr_config& cfg, int n_out, bool fx);
// workgroups of the persistent launch: as many as fit on every CU at once with
// n_out per-splat outputs staged per entry
int persistent_grid(const potr_config& cfg, int n_out, bool fx);
potr_status launch_render_score(const ViewJobs& jobs, int32_t n_views, int32_t tiles_per_view,
                                const potr_config& cfg, bool fx, hipStream_t s);
// out[i] = acc[i] * 2^-32 (fixed-point sums to FP32)
potr_status launch_fixed_to_float(int64_t n, const int64_t* acc, float* out, hipStream_t s);
// with_se: some job of the table has scores_se (the kernel then also keeps the
// per-entry dSE sums; jobs without it skip them); n_out: the most per-splat
// outputs (1..3) any job of the table has, which sizes the LDS
potr_status launch_render_score_persistent(const ViewJob* jobs_dev, int32_t n_jobs, const int64_t* item_prefix_dev,
                                           int64_t* counter_dev, int32_t grid, const potr_config& cfg,
                                           bool with_se, int n_out, bool fx, hipStream_t s);

}  // namespace potr
