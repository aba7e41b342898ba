// C ABI of libpotr.so: argument validation, workspace sizing, error reporting.
// Every entry point validates on the host, then enqueues kernels on the
// caller's stream; none of them allocates device memory.
#include <hip/hip_runtime.h>

#include <cstdarg>
#include <cstdio>
#include <cstring>

#include "common.h"
#include "fused.h"
#include "prune.h"
#include "sh_compact.h"

namespace potr {

static thread_local char g_err[512] = "";

potr_status fail(potr_status st, const char* fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
    return st;
}

potr_status check_launch(const char* what) {
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(POTR_EHIP, "%s: %s", what, hipGetErrorString(e));
    return POTR_OK;
}

}  // namespace potr

using namespace potr;

namespace {

potr_status check_cfg(const potr_config* cfg) {
    if (!cfg) return fail(POTR_EINVAL, "config is NULL");
    const bool shape_ok = (cfg->tile_w == 16 && cfg->tile_h == 16) || (cfg->tile_w == 8 && cfg->tile_h == 8) ||
                          (cfg->tile_w == 32 && cfg->tile_h == 8);
    if (!shape_ok) return fail(POTR_EINVAL, "tile %dx%d: expected 16x16, 8x8 or 32x8", cfg->tile_w, cfg->tile_h);
    if (cfg->lds_batch < 64 || cfg->lds_batch > 512 || cfg->lds_batch % 64)
        return fail(POTR_EINVAL, "lds_batch %d: expected 64..512, multiple of 64", cfg->lds_batch);
    if (cfg->sh_degree < 0 || cfg->sh_degree > 3) return fail(POTR_EINVAL, "sh_degree %d not in 0..3", cfg->sh_degree);
    if (!(cfg->alpha_min > 0.f) || !(cfg->alpha_max < 1.f) || !(cfg->alpha_min <= cfg->alpha_max))
        return fail(POTR_EINVAL, "need 0 < alpha_min <= alpha_max < 1");
    if (!(cfg->q_max > 0.f) || !(cfg->t_min >= 0.f) || !(cfg->t_min < 1.f) || !(cfg->eps2d >= 0.f))
        return fail(POTR_EINVAL, "need q_max > 0, 0 <= t_min < 1, eps2d >= 0");
    return POTR_OK;
}

potr_status check_cams(int32_t V, const potr_camera* cams, const potr_config* cfg) {
    if (V < 1) return fail(POTR_EINVAL, "V = %d, need >= 1", V);
    if (!cams) return fail(POTR_EINVAL, "cams is NULL");
    for (int32_t v = 0; v < V; ++v) {
        const potr_camera& c = cams[v];
        if (c.width < 1 || c.height < 1 || c.width > 16384 || c.height > 16384)
            return fail(POTR_EINVAL, "view %d: size %dx%d out of range", v, c.width, c.height);
        if (c.width != cams[0].width || c.height != cams[0].height)
            return fail(POTR_EINVAL, "view %d: all views of one call need the same size", v);
        if (!(c.fx > 0.f) || !(c.fy > 0.f)) return fail(POTR_EINVAL, "view %d: focal lengths must be > 0", v);
    }
    const int64_t tiles = (int64_t)tiles_x(cams[0], *cfg) * tiles_y(cams[0], *cfg);
    if (tiles * V >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "too many tiles x views");
    return POTR_OK;
}

bool aligned16(const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15u) == 0; }

}  // namespace

extern "C" {

int32_t potr_abi_version(void) { return POTR_ABI_VERSION; }

const char* potr_last_error(void) { return g_err; }

potr_status potr_project(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg, const float* means,
                         const float* scales, const float* quats, const float* opac, const float* sh,
                         potr_proj* proj, int32_t* tiles_touched, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld out of range", (long long)N);
    if (N > 0 && (!means || !scales || !quats || !opac || !sh || !proj || !tiles_touched))
        return fail(POTR_EINVAL, "NULL buffer");
    if (!aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    if (N > 0 && !aligned16(sh)) return fail(POTR_EINVAL, "sh must be 16-byte aligned");
    return launch_project(N, V, cams, *cfg, means, scales, quats, opac, sh, proj, tiles_touched,
                          (hipStream_t)stream);
}

potr_status potr_bin_workspace_size(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                    size_t* bytes) {
    if (!bytes || N < 0) return fail(POTR_EINVAL, "bad arguments");
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    *bytes = bin_workspace_bytes(N, V, tiles_x(cams[0], *cfg), tiles_y(cams[0], *cfg));
    return POTR_OK;
}

potr_status potr_bin(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg, const potr_proj* proj,
                     void* ws, size_t ws_bytes, uint32_t* order, int64_t* n_pairs, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0 || N * (int64_t)V >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N x V out of range");
    if (!n_pairs || !ws || (N > 0 && (!proj || !order))) return fail(POTR_EINVAL, "NULL buffer");
    if (N > 0 && !aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    const size_t need = bin_workspace_bytes(N, V, tiles_x(cams[0], *cfg), tiles_y(cams[0], *cfg));
    if (ws_bytes < need) return fail(POTR_ECAPACITY, "bin workspace %zu < %zu bytes", ws_bytes, need);
    return launch_bin(N, V, cams[0], *cfg, proj, ws, order, n_pairs, (hipStream_t)stream);
}

potr_status potr_sort_workspace_size(int64_t capacity, size_t* bytes) {
    if (!bytes || capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "bad arguments");
    *bytes = sort_workspace_bytes(capacity);
    return POTR_OK;
}

potr_status potr_sort(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg, const potr_proj* proj,
                      const uint32_t* order, void* ws, size_t ws_bytes, const int64_t* n_pairs, int64_t capacity,
                      void* sort_ws, size_t sort_ws_bytes, uint32_t* sorted_ids, int32_t* tile_ranges,
                      void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0 || N * (int64_t)V >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N x V out of range");
    if (capacity < 0 || capacity >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "capacity out of range");
    if (!n_pairs || !ws || !tile_ranges || !sort_ws || (N > 0 && (!proj || !order)) || (capacity > 0 && !sorted_ids))
        return fail(POTR_EINVAL, "NULL buffer");
    const size_t need = bin_workspace_bytes(N, V, tiles_x(cams[0], *cfg), tiles_y(cams[0], *cfg));
    if (ws_bytes < need) return fail(POTR_ECAPACITY, "bin workspace %zu < %zu bytes", ws_bytes, need);
    if (sort_ws_bytes < sort_workspace_bytes(capacity))
        return fail(POTR_ECAPACITY, "sort workspace %zu < %zu bytes", sort_ws_bytes, sort_workspace_bytes(capacity));
    return launch_sort(N, V, cams[0], *cfg, proj, order, ws, n_pairs, capacity, sort_ws, sorted_ids, tile_ranges,
                       (hipStream_t)stream);
}

potr_status potr_blend(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                       const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges, float* image,
                       float* p_final, float* t_final, int32_t* n_walk, int32_t* n_blend, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (!tile_ranges || !image || (N > 0 && (!proj || !sorted_ids))) return fail(POTR_EINVAL, "NULL buffer");
    if (!aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    return launch_blend(N, V, cams[0], *cfg, proj, sorted_ids, tile_ranges, image, p_final, t_final, n_walk,
                        n_blend, (hipStream_t)stream);
}

potr_status potr_score(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                       const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                       const float* p_final, const float* t_final, const int32_t* n_walk, const float* target,
                       float* scores, float* scores_se, float* importance, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (N == 0) return POTR_OK;   /* no splat: nothing to accumulate */
    if (!tile_ranges || !p_final || !t_final || !n_walk || !proj || !sorted_ids)
        return fail(POTR_EINVAL, "NULL buffer");
    if (scores_se && !target) return fail(POTR_EINVAL, "scores_se needs a target image");
    if (!scores && !scores_se && !importance) return fail(POTR_EINVAL, "no output requested");
    if (!aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    return launch_score(N, V, cams[0], *cfg, proj, sorted_ids, tile_ranges, p_final, t_final, n_walk, target,
                        scores, scores_se, importance, (hipStream_t)stream);
}

potr_status potr_blend_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                                const float* p_final, const float* t_final, const int32_t* n_walk,
                                const float* dL_dimage, float* grad2d, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (N == 0) return POTR_OK;
    if (!proj || !sorted_ids || !tile_ranges || !p_final || !t_final || !n_walk || !dL_dimage || !grad2d)
        return fail(POTR_EINVAL, "NULL buffer");
    if (!aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    return launch_blend_backward(N, V, cams[0], *cfg, proj, sorted_ids, tile_ranges, p_final, t_final, n_walk,
                                 dL_dimage, grad2d, (hipStream_t)stream);
}

potr_status potr_project_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                  const float* means, const float* scales, const float* quats, const float* opac,
                                  const float* sh, const float* grad2d, float* d_means, float* d_scales,
                                  float* d_quats, float* d_opac, float* d_sh, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld out of range", (long long)N);
    if (N == 0) return POTR_OK;
    if (!means || !scales || !quats || !opac || !sh || !grad2d || !d_means || !d_scales || !d_quats || !d_opac ||
        !d_sh)
        return fail(POTR_EINVAL, "NULL buffer");
    return launch_project_backward(N, V, cams, *cfg, means, scales, quats, opac, sh, grad2d, d_means, d_scales,
                                   d_quats, d_opac, d_sh, (hipStream_t)stream);
}

potr_status potr_backward_workspace_size(int64_t N, int32_t V, size_t* bytes) {
    if (!bytes || N < 0 || V < 1) return fail(POTR_EINVAL, "bad arguments");
    *bytes = (size_t)N * V * 9 * sizeof(float);
    return POTR_OK;
}

potr_status potr_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                          const float* means, const float* scales, const float* quats, const float* opac,
                          const float* sh, const potr_proj* proj, const uint32_t* sorted_ids,
                          const int32_t* tile_ranges, const float* p_final, const float* t_final,
                          const int32_t* n_walk, const float* dL_dimage, void* ws, size_t ws_bytes,
                          float* d_means, float* d_scales, float* d_quats, float* d_opac, float* d_sh,
                          void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0 || N * (int64_t)V >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N x V out of range");
    if (N == 0) return POTR_OK;
    if (!ws) return fail(POTR_EINVAL, "NULL workspace");
    if (ws_bytes < (size_t)N * V * 9 * sizeof(float))
        return fail(POTR_ECAPACITY, "backward workspace %zu < %zu bytes", ws_bytes, (size_t)N * V * 9 * sizeof(float));
    float* g2 = (float*)ws;
    st = launch_zero(g2, N * V * 9, (hipStream_t)stream);
    if (st == POTR_OK)
        st = potr_blend_backward(N, V, cams, cfg, proj, sorted_ids, tile_ranges, p_final, t_final, n_walk, dL_dimage,
                                 g2, stream);
    if (st == POTR_OK)
        st = potr_project_backward(N, V, cams, cfg, means, scales, quats, opac, sh, g2, d_means, d_scales, d_quats,
                                   d_opac, d_sh, stream);
    return st;
}

potr_status potr_render_score_out(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                  const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                                  float* image, const float* target, const potr_outputs* out, void* stream) {
    potr_status st = check_cfg(cfg);
    if (st == POTR_OK) st = check_cams(V, cams, cfg);
    if (st != POTR_OK) return st;
    if (N < 0) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (!out) return fail(POTR_EINVAL, "NULL outputs");
    st = check_outputs(*out, N, V, target);
    if (st != POTR_OK) return st;
    if (!tile_ranges || (N > 0 && (!proj || !sorted_ids))) return fail(POTR_EINVAL, "NULL buffer");
    if (!image && !out->scores && !out->scores_se && !out->importance) return fail(POTR_EINVAL, "no output requested");
    if (!aligned16(proj)) return fail(POTR_EINVAL, "proj must be 16-byte aligned");
    const potr_camera& c = cams[0];
    const int tx = tiles_x(c, *cfg), T = tx * tiles_y(c, *cfg);
    const int64_t P = (int64_t)c.width * c.height;
    for (int32_t v0 = 0; v0 < V; v0 += kViewsPerLaunch) {
        const int32_t nv = V - v0 < kViewsPerLaunch ? V - v0 : kViewsPerLaunch;
        ViewJobs jobs{};
        for (int32_t k = 0; k < nv; ++k) {
            ViewJob& j = jobs.j[k];
            const int64_t v = v0 + k;
            j.proj = proj + v * N;
            j.ids = sorted_ids;
            j.ranges = tile_ranges + v * T * 2;
            j.W = c.width;
            j.H = c.height;
            j.tiles_x = tx;
            j.tiles = T;
            j.image = image ? image + v * P * 3 : nullptr;
            j.target = target ? target + v * P * 3 : nullptr;
            set_outputs(j, *out, N, v);
        }
        st = launch_render_score(jobs, nv, T, *cfg, out->fixed_point != 0, (hipStream_t)stream);
        if (st != POTR_OK) return st;
    }
    return POTR_OK;
}

potr_status potr_fixed_to_float(const int64_t* acc, int64_t n, float* out, void* stream) {
    if (n < 0 || (n > 0 && (!acc || !out))) return fail(POTR_EINVAL, "bad argument");
    return launch_fixed_to_float(n, acc, out, (hipStream_t)stream);
}

potr_status potr_render_score(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                              const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                              float* image, const float* target, float* scores, float* scores_se, float* importance,
                              void* stream) {
    potr_outputs o{};
    o.scores = scores;
    o.scores_se = scores_se;
    o.importance = importance;
    o.scores_weight = o.se_weight = o.importance_weight = 1.f;
    return potr_render_score_out(N, V, cams, cfg, proj, sorted_ids, tile_ranges, image, target, &o, stream);
}

potr_status potr_prune_workspace_size(int64_t N, size_t* bytes) {
    if (!bytes || N < 0) return fail(POTR_EINVAL, "bad argument");
    const size_t a = prune_select_scratch_bytes(), b = prune_compact_scratch_bytes(N);
    *bytes = a > b ? a : b;
    return POTR_OK;
}

potr_status potr_prune_select(int64_t N, const float* dmse, const float* importance, double dmse_max,
                              int32_t remaining, double a, void* ws, size_t ws_bytes, uint8_t* remove,
                              int64_t* n_removed, void* stream) {
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (!(dmse_max > 0.0) || dmse_max > 1e300) return fail(POTR_EINVAL, "dmse_max = %g", dmse_max);
    if (!(a > 0.0) || a > 1e300) return fail(POTR_EINVAL, "a = %g", a);
    if (remaining < 1) return fail(POTR_EINVAL, "remaining = %d", remaining);
    if (!ws || !n_removed || (N > 0 && (!dmse || !importance || !remove))) return fail(POTR_EINVAL, "NULL buffer");
    if (ws_bytes < prune_select_scratch_bytes()) return fail(POTR_ECAPACITY, "prune workspace %zu bytes", ws_bytes);
    return launch_prune_select(N, dmse, importance, dmse_max, remaining, a, ws, remove, n_removed,
                               (hipStream_t)stream);
}

potr_status potr_sh_compact_workspace_size(int64_t N, int32_t V, size_t* bytes) {
    if (!bytes || N < 0 || V < 1) return fail(POTR_EINVAL, "bad argument");
    *bytes = sh_compact_workspace_bytes(N, V);
    return POTR_OK;
}

potr_status potr_sh_compact(int64_t N, int32_t V, const potr_camera* cams, int32_t sh_degree, const float* means,
                            const float* sh, const float* importance, int64_t importance_stride, double lam,
                            double alpha, double tau, void* ws, size_t ws_bytes, float* sh_out, void* stream) {
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (V < 1 || !cams) return fail(POTR_EINVAL, "need at least one camera");
    if (sh_degree < 0 || sh_degree > 3) return fail(POTR_EINVAL, "sh_degree %d not in 0..3", sh_degree);
    if (!(lam >= 0.0) || lam > 1e300 || !(alpha >= 0.0) || alpha > 1e300 || !(tau >= 0.0) || tau > 1e300)
        return fail(POTR_EINVAL, "lam, alpha, tau must be finite and >= 0");
    if (importance_stride < N) return fail(POTR_EINVAL, "importance stride %lld < N", (long long)importance_stride);
    if (!ws || (N > 0 && (!means || !sh || !importance || !sh_out))) return fail(POTR_EINVAL, "NULL buffer");
    if (N > 0 && sh_out < sh + 48 * N && sh < sh_out + 48 * N) return fail(POTR_EINVAL, "sh_out overlaps sh");
    if (ws_bytes < sh_compact_workspace_bytes(N, V))
        return fail(POTR_ECAPACITY, "SH compaction workspace %zu < %zu bytes", ws_bytes,
                    sh_compact_workspace_bytes(N, V));
    if (!aligned16(ws)) return fail(POTR_EINVAL, "workspace must be 16-byte aligned");
    const ShCompactParams p{lam, alpha, tau};
    return launch_sh_compact(N, V, cams, sh_degree, means, sh, importance, importance_stride, p, ws, sh_out,
                             (hipStream_t)stream);
}

potr_status potr_prune_select_noalloc(int64_t N, const float* dmse, const float* importance, double dmse_max,
                                      int32_t remaining, double a, uint8_t* remove, int64_t* n_removed,
                                      void* stream) {
    if (N < 0 || N >= (int64_t(1) << 31))
        return fail(POTR_EINVAL, "N = %lld: the no-allocation select takes at most 2^31 - 1 splats", (long long)N);
    if (!(dmse_max > 0.0) || dmse_max > 1e300) return fail(POTR_EINVAL, "dmse_max = %g", dmse_max);
    if (!(a > 0.0) || a > 1e300) return fail(POTR_EINVAL, "a = %g", a);
    if (remaining < 1) return fail(POTR_EINVAL, "remaining = %d", remaining);
    if (!n_removed || (N > 0 && (!dmse || !importance || !remove))) return fail(POTR_EINVAL, "NULL buffer");
    return launch_prune_select_noalloc(N, dmse, importance, dmse_max, remaining, a, remove, n_removed,
                                       (hipStream_t)stream);
}

potr_status potr_prune_compact(int64_t N, const uint8_t* remove, const float* means, const float* scales,
                               const float* quats, const float* opac, const float* sh, const int32_t* ids, void* ws,
                               size_t ws_bytes, float* means_out, float* scales_out, float* quats_out,
                               float* opac_out, float* sh_out, int32_t* ids_out, int64_t* n_kept, void* stream) {
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (!ws || !n_kept) return fail(POTR_EINVAL, "NULL buffer");
    if (N > 0 && (!remove || !means || !scales || !quats || !opac || !sh || !means_out || !scales_out ||
                  !quats_out || !opac_out || !sh_out || !ids_out))
        return fail(POTR_EINVAL, "NULL buffer");
    if (!aligned16(quats) || !aligned16(sh) || !aligned16(quats_out) || !aligned16(sh_out))
        return fail(POTR_EINVAL, "quats and sh must be 16-byte aligned");
    if (ws_bytes < prune_compact_scratch_bytes(N)) return fail(POTR_ECAPACITY, "prune workspace %zu bytes", ws_bytes);
    const PruneArrays in{means, scales, quats, opac, sh, ids};
    const PruneOut out{means_out, scales_out, quats_out, opac_out, sh_out, ids_out};
    return launch_prune_compact(N, remove, in, out, ws, n_kept, (hipStream_t)stream);
}

}  // extern "C"
