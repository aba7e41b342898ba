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
    float* scores;            // [N] += sum |PD|_1, or null
    float* importance;        // [N] += sum T alpha, or null
    float* scores_se;         // [N] += sum dSE, or null
};

struct ViewJobs {
    ViewJob j[kViewsPerLaunch];
};

// dynamic LDS bytes of the fused pass with n_out per-splat outputs
size_t fused_smem_bytes(const potr_config& cfg, int n_out);
int persistent_grid(const potr_config& cfg);
potr_status launch_render_score(const ViewJobs& jobs, int32_t n_views, int32_t tiles_per_view,
                                const potr_config& cfg, hipStream_t s);
potr_status launch_render_score_persistent(const ViewJob* jobs_dev, int32_t n_jobs, const int64_t* item_prefix_dev,
                                           int64_t* counter_dev, int32_t grid, const potr_config& cfg,
                                           hipStream_t s);

}  // namespace potr
