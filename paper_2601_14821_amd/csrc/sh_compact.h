// SH energy compaction (paper Sec. 4.4).
#pragma once

#include "common.h"

namespace potr {

struct ShCompactParams {
    double lam;     // ridge coefficient of the luminance channel (chrominance: 3 lam)
    double alpha;   // |cosine| above which an AC column counts as parallel to a kept one
    double tau;     // first-pass AC coefficients below this are forced to zero
};

size_t sh_compact_workspace_bytes(int64_t N, int32_t V);
potr_status launch_sh_compact(int64_t N, int32_t V, const potr_camera* cams, int degree, const float* means,
                              const float* sh, const float* imp, int64_t stride, const ShCompactParams& p,
                              void* ws, float* sh_out, hipStream_t s);

}  // namespace potr
