// Internal declarations shared by the HIP translation units of libpotr.so.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "potr.h"

namespace potr {

// Views whose cameras travel by value in one launch's kernel arguments.
constexpr int kViewsPerLaunch = 32;

struct CamBatch {
    potr_camera c[kViewsPerLaunch];
};

inline int tiles_x(const potr_camera& c, const potr_config& g) { return (c.width + g.tile_w - 1) / g.tile_w; }
inline int tiles_y(const potr_camera& c, const potr_config& g) { return (c.height + g.tile_h - 1) / g.tile_h; }

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }
inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// Thread-local error text behind potr_last_error().
potr_status fail(potr_status st, const char* fmt, ...);
// Turns the last launch error on this thread into POTR_EHIP.
potr_status check_launch(const char* what);

// ---- launchers (defined in the .hip files) ----
struct BinKeys;
// keys (optional): also write the bin's keys, rects and key-range partials there;
// tiles_touched may be NULL (not written)
potr_status launch_project(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                           const float* means, const float* scales, const float* quats, const float* opac,
                           const float* sh, potr_proj* proj, int32_t* tiles_touched, hipStream_t s,
                           const BinKeys* keys = nullptr);

size_t bin_workspace_bytes(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y);
// Where a projection launch can write, in a bin workspace, what the bin's first
// kernel would otherwise take from the records: per (view, splat) the depth key
// (its FP32 bits) and the packed rect (x0 | x1 << 16, y0 | y1 << 16), and per
// (view, wave of 64 splats) the wave's largest key and largest complemented key.
struct BinKeys {
    uint32_t* keys;
    uint2* rects;
    uint2* part;
    int64_t per_view;   // partials per view: ceil(N / 64)
};
BinKeys bin_keys(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg, void* ws);
// keys_ready: the launch_project before this call wrote bin_keys(...) of this workspace
potr_status launch_bin(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                       const potr_proj* proj, void* ws, uint32_t* order, int64_t* n_pairs, hipStream_t s,
                       bool keys_ready = false);
size_t sort_workspace_bytes(int64_t capacity);
potr_status launch_sort(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                        const potr_proj* proj, const uint32_t* order, void* ws, const int64_t* n_pairs,
                        int64_t capacity, void* sort_ws, uint32_t* sorted_ids, int32_t* tile_ranges,
                        hipStream_t s);

potr_status launch_blend(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                         const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                         float* image, float* p_final, float* t_final, int32_t* n_walk, int32_t* n_blend,
                         hipStream_t s);

potr_status launch_score(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                         const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                         const float* p_final, const float* t_final, const int32_t* n_walk,
                         const float* target, float* scores, float* scores_se, float* importance,
                         hipStream_t s);

potr_status launch_blend_backward(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                                  const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                                  const float* p_final, const float* t_final, const int32_t* n_walk,
                                  const float* dL_dimage, float* grad2d, hipStream_t s);
potr_status launch_project_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                                    const float* means, const float* scales, const float* quats, const float* opac,
                                    const float* sh, const float* grad2d, float* d_means, float* d_scales,
                                    float* d_quats, float* d_opac, float* d_sh, hipStream_t s);
potr_status launch_zero(float* p, int64_t n, hipStream_t s);

}  // namespace potr
