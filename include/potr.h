/*
 * potr.h -- C ABI of libpotr.so, the MI355X (gfx950) removal-effect rasterizer.
 *
 * The library computes, for every splat of a 3D Gaussian splatting scene and every
 * view, the change of every pixel's colour if that splat alone were deleted
 * (POTR, "Post-Training 3DGS Compression", Sec. 4.2: the pruning difference
 * PD_k(x) = c~_k(x) - c(x)), and reduces it per splat. Its stages follow the
 * forward rendering of Sec. 3: projection of each 3D Gaussian to a 2D Gaussian by
 * an affine approximation, colour from real spherical harmonics, ordering of the
 * splats by approximate depth, front-to-back alpha compositing
 * (T_k = prod_{j<k} (1 - alpha_j), c = sum_k T_k alpha_k c_k + T_K bg).
 *
 * Conventions shared by all calls
 *  - Every pointer is a DEVICE pointer unless marked (host). The caller owns all
 *    memory; the library never allocates or frees caller buffers.
 *  - `stream` is a hipStream_t (NULL = the null stream). Calls only enqueue work
 *    on it and return; results are ready when the stream is synchronised.
 *  - Splat parameters (FP32, row per splat, 236 bytes per splat):
 *      means [N,3], scales [N,3] (activated, > 0), quats [N,4] (w,x,y,z; any norm,
 *      zero norm culls), opac [N] (activated, in (0,1)), sh [N,16,3] (real SH
 *      coefficients, coefficient-major, index l(l+1)+m).
 *  - Images are [V,H,W,3] FP32, pixel (i,j) sampled at (i+0.5, j+0.5).
 *  - Every view of one call has the same width and height.
 *  - Errors: a negative potr_status; potr_last_error() returns a message for the
 *    calling thread. Validation errors (POTR_EINVAL) are raised before any launch.
 *    POTR_EHIP carries the HIP runtime's message.
 *  - Calls on distinct streams may run concurrently; calls sharing a workspace on
 *    one stream must not overlap.
 */
#ifndef POTR_H
#define POTR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define POTR_ABI_VERSION 3

#define POTR_API __attribute__((visibility("default")))

typedef int32_t potr_status;
#define POTR_OK 0
#define POTR_EINVAL (-1)        /* bad argument; nothing was launched */
#define POTR_ECAPACITY (-2)     /* a caller buffer is too small (see potr_bin) */
#define POTR_EHIP (-3)          /* HIP runtime error */
#define POTR_EUNSUPPORTED (-4)  /* valid request this build does not handle */

/* Pinhole camera, OpenCV axes (x right, y down, z forward). R (row-major) and t
 * map world points to camera coordinates: p_cam = R p + t. */
typedef struct potr_camera {
    float R[9];
    float t[3];
    float fx, fy, cx, cy;
    int32_t width, height;
} potr_camera;

/* Rasterizer settings. Where the paper leaves a detail open, the setting names it.
 *  tile_w x tile_h : screen tile, one of 16x16, 8x8, 32x8
 *  lds_batch       : splat records staged in LDS per batch, 64..512, multiple of 64
 *  eps2d           : low-pass added to the 2D covariance diagonal (px^2), e.g. 0.3
 *  near_z          : splats with camera z <= near_z are culled
 *  jclamp          : x/z and y/z in the Jacobian are clamped to +-jclamp half fields of view
 *  alpha_min       : a splat counts at a pixel only if o*exp(-q/2) >= alpha_min (e.g. 1/255)
 *  alpha_max       : alpha = min(alpha_max, o*exp(-q/2)) (e.g. 0.99)
 *  q_max           : a splat counts at a pixel only if its Mahalanobis q <= q_max (e.g. 9)
 *  t_min           : compositing stops before the splat that would drive the
 *                    transmittance below t_min (e.g. 1e-4); 0 = exact mode, no stop
 *  bg              : background colour, entering as T_final * bg
 *  sh_degree       : 0..3 */
typedef struct potr_config {
    int32_t tile_w, tile_h;
    int32_t lds_batch;
    float eps2d, near_z, jclamp;
    float alpha_min, alpha_max, q_max, t_min;
    float bg[3];
    int32_t sh_degree;
} potr_config;

/* Projected splat for one view (48 bytes). Culled splats have opacity 0 and an
 * empty rect.
 *  mean2d : centre in pixels
 *  conic  : inverse 2D covariance (a, b, c): q = a dx^2 + 2 b dx dy + c dy^2
 *  opacity: base opacity o
 *  rgb    : colour, max(0, sum_i L_i Y_i(d) + 1/2), d from the camera centre to the splat
 *  depth  : camera z by the fixed FP32 chain fma(R22,z,fma(R21,y,fma(R20,x,t_z)));
 *           its bit pattern orders the splats of a view
 *  rect   : tiles x0, y0, x1, y1 (half-open) that can hold a pixel where the splat
 *           counts; a conservative bound, so images do not depend on the tile shape */
typedef struct potr_proj {
    float mean2d[2];
    float conic[3];
    float opacity;
    float rgb[3];
    float depth;
    int16_t rect[4];
} potr_proj;

POTR_API int32_t potr_abi_version(void);
POTR_API const char* potr_last_error(void);

/* ---------------------------------------------------------------------------
 * potr_project -- Sec. 3: affine (Jacobian) projection of each 3D Gaussian,
 * Sigma' = J W Sigma W^T J^T + eps2d I with Sigma = R(q) diag(s^2) R(q)^T, its
 * inverse (the conic), the SH colour along the camera-to-centre direction, the
 * depth key and the tile rectangle, for N splats x V views.
 *   cams  (host) [V]
 *   sh    [N,16,3] FP32, 16-byte aligned (read as float4)
 *   proj  [V*N] potr_proj, view-major (proj[v*N + i])
 *   tiles_touched [V*N] int32: number of tiles in rect (0 if culled)
 * Arithmetic: the projection runs in FP64 and stores FP32.
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_project(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                         const float* means, const float* scales, const float* quats,
                         const float* opac, const float* sh,
                         potr_proj* proj, int32_t* tiles_touched, void* stream);

/* ---------------------------------------------------------------------------
 * potr_bin -- Sec. 3 ("layers ordered by approximate depth"): order each view's
 * splats by depth key (ties by splat id) and count the (tile, splat) pairs:
 * every tile of a splat's rect holds the splat. The counts per group of 4096
 * consecutive depth ranks and tile, and per group and row of tiles, their
 * offsets, and the rects in depth order are kept in the workspace for
 * potr_sort, which only reads it (so potr_sort may be called again, e.g. with
 * a larger capacity, without binning again).
 *   proj   [V*N] from potr_project, 16-byte aligned (its depth keys and rects are read)
 *   ws     workspace of potr_bin_workspace_size bytes; potr_sort reads it, so
 *          it must stay untouched between the two calls
 *   order  [V*N] uint32 out: order[v*N + r] = id of the splat with depth rank r in view v
 *   n_pairs (device) int64 out: total number of pairs over all views
 * Cost: the workspace holds 32 bytes per (view, splat) (depth sort keys and
 * values, rects by id and in depth order), 8 bytes per (view, group of 4096
 * ranks, tile) and 8 bytes per (view, group, tile row).
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_bin_workspace_size(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                    size_t* bytes);
POTR_API potr_status potr_bin(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                     const potr_proj* proj, void* ws, size_t ws_bytes, uint32_t* order, int64_t* n_pairs,
                     void* stream);

/* ---------------------------------------------------------------------------
 * potr_sort -- each tile's list of splat ids in (depth key, splat id) order,
 * all tiles of all views back to back in (view, tile) order: the order a sort
 * of (view, tile, depth, id) keys gives, obtained by placing every pair
 * directly from the counts potr_bin left in its workspace (no per-pair sort):
 * first every group's list of the splats covering each tile row, in rank
 * order (into sort_ws), then per (group of 4096 ranks, tile row) the list's
 * pairs at their tiles' offsets.
 * N, V, cams, cfg, proj, order and ws are those of the potr_bin call before
 * (ws is read, not changed, so potr_sort may be called again, e.g. with a
 * larger capacity).
 *   n_pairs  (device) from potr_bin
 *   capacity (host) number of slots in sorted_ids; with more pairs than that
 *            nothing is placed and every range is empty (grow and call again)
 *   sort_ws  workspace of potr_sort_workspace_size(capacity) bytes: the row
 *            lists, 8 bytes per (splat, covered tile row), at most one per pair
 *   sorted_ids [capacity] uint32 out: splat id (0..N-1) of every pair
 *   tile_ranges [V*tiles*2] int32 out: half-open [start, end) into sorted_ids;
 *            [0, 0) for a tile without pairs
 * Limits: every image the camera checks accept (at most 16384 px a side, so
 * up to 2048 tile columns of 8 px) fits the per-workgroup LDS (72.0 KB at 2048
 * columns).
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_sort_workspace_size(int64_t capacity, size_t* bytes);
POTR_API potr_status potr_sort(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                      const potr_proj* proj, const uint32_t* order, void* ws, size_t ws_bytes,
                      const int64_t* n_pairs, int64_t capacity, void* sort_ws, size_t sort_ws_bytes,
                      uint32_t* sorted_ids, int32_t* tile_ranges, void* stream);

/* ---------------------------------------------------------------------------
 * potr_blend -- Sec. 3, eq. (alpha_blending): front-to-back compositing per pixel
 * over its tile's sorted list.
 *   image   [V,H,W,3] out: P_K + T_final * bg
 *   p_final [V,H,W,3] out: P_K = sum_k T_k alpha_k c_k (paper's partial colour after K splats)
 *   t_final [V,H,W]   out: T after the last blended splat
 *   n_walk  [V,H,W]   out int32: list entries visited before the stop (or the list length)
 *   n_blend [V,H,W]   out int32 or NULL: splats blended (K)
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_blend(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                       const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                       float* image, float* p_final, float* t_final, int32_t* n_walk, int32_t* n_blend,
                       void* stream);

/* ---------------------------------------------------------------------------
 * potr_score -- Sec. 4.2: the pruning difference of every blended splat k at every
 * pixel, PD_k = -c_k alpha_k T_k + alpha_k/(1-alpha_k) (S_k + T_final bg) with
 * S_k = P_K - P_{k+1} (equal to the paper's partial-colour form), reduced per splat
 * over pixels and views. Outputs are ACCUMULATED (+=); zero them first.
 *   scores     [N] += sum over pixels and channels of |PD_k|         (may be NULL)
 *   scores_se  [N] += sum over pixels and channels of dSE_k
 *                     = |PD_k|^2 + 2 PD_k.(c - target)  (Sec. 4.2; needs target)
 *   importance [N] += sum over pixels of T_k alpha_k  (Sec. 4.1, before the 1/P)
 *   target     [V,H,W,3] or NULL
 * Inputs p_final, t_final, n_walk come from potr_blend with the same lists.
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_score(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                       const potr_proj* proj, const uint32_t* sorted_ids, const int32_t* tile_ranges,
                       const float* p_final, const float* t_final, const int32_t* n_walk,
                       const float* target, float* scores, float* scores_se, float* importance,
                       void* stream);

/* ---------------------------------------------------------------------------
 * Backward of the forward render for a loss L given dL/dimage [V,H,W,3]: the
 * standard training pass that the paper's fine-tuning stage runs (Sec. 4.6).
 * With S_k = P_K - P_{k+1} per pixel,
 *   dC/dc_k = T_k alpha_k,  dC/dalpha_k = T_k c_k - (S_k + T_final bg)/(1 - alpha_k),
 * alpha_k = min(alpha_max, o G), G = exp(-q/2) (no gradient through the clamp,
 * the colour clamp at 0 or the Jacobian clamp). The removal effect of Sec. 4.2
 * is PD_k = -alpha_k dC/dalpha_k.
 *
 * potr_blend_backward: grad2d [V*N*9] += per (view, splat):
 *   d mean2d.x, d mean2d.y, d conic.a, d conic.b, d conic.c, d opacity, d r, d g, d b
 *   (conic.b is the stored off-diagonal entry, entering q as 2b dx dy).
 * potr_project_backward: chains grad2d through the projection (FP64) into
 *   d_means [N,3], d_scales [N,3], d_quats [N,4] (w.r.t. the unnormalised
 *   quaternion), d_opac [N], d_sh [N,16,3]; all ACCUMULATED (+=), summed over views.
 * potr_backward: both, with grad2d in a workspace of potr_backward_workspace_size
 *   bytes that it clears itself.
 * Inputs proj, sorted_ids, tile_ranges, p_final, t_final, n_walk are those of
 * the forward (potr_project ... potr_blend) of the same views.
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_blend_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                         const potr_proj* proj, const uint32_t* sorted_ids,
                                         const int32_t* tile_ranges, const float* p_final, const float* t_final,
                                         const int32_t* n_walk, const float* dL_dimage, float* grad2d, void* stream);
POTR_API potr_status potr_project_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                           const float* means, const float* scales, const float* quats,
                                           const float* opac, const float* sh, const float* grad2d,
                                           float* d_means, float* d_scales, float* d_quats, float* d_opac,
                                           float* d_sh, void* stream);
POTR_API potr_status potr_backward_workspace_size(int64_t N, int32_t V, size_t* bytes);
POTR_API potr_status potr_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                   const float* means, const float* scales, const float* quats, const float* opac,
                                   const float* sh, const potr_proj* proj, const uint32_t* sorted_ids,
                                   const int32_t* tile_ranges, const float* p_final, const float* t_final,
                                   const int32_t* n_walk, const float* dL_dimage, void* ws, size_t ws_bytes,
                                   float* d_means, float* d_scales, float* d_quats, float* d_opac, float* d_sh,
                                   void* stream);

/* ---------------------------------------------------------------------------
 * potr_render_score -- potr_blend and potr_score fused in one launch per view
 * batch: each tile is composited front to back and its walked prefix revisited
 * for the removal effect, reusing the LDS-staged records. Same per-pixel
 * arithmetic as the two calls: the image is bit-identical to potr_blend's, the
 * per-splat sums equal up to the order of their float additions (over a tile's
 * waves in LDS, over tiles and views in device atomics). image may be NULL;
 * scores, importance, scores_se as in potr_score (+=; at least one non-NULL;
 * scores_se needs target).
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_render_score(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                       const potr_proj* proj, const uint32_t* sorted_ids,
                                       const int32_t* tile_ranges, float* image, const float* target,
                                       float* scores, float* scores_se, float* importance, void* stream);

/* ---------------------------------------------------------------------------
 * potr_outputs -- where the fused pass and the batch put their per-splat
 * reductions (Sec. 4.1 importance, Sec. 4.2 removal effect and dSE), each one
 * optional (NULL):
 *   scores      sum over pixels and channels of |PD_k|
 *   scores_se   sum over pixels and channels of dSE_k = |PD_k|^2 + 2 PD_k.(c - c_t)
 *               (needs a target image c_t)
 *   importance  sum over pixels of T_k alpha_k
 * For view v of a call, output o lives at o + v * o_stride: stride 0 adds every
 * view into one [N] array, stride N gives one [N] array per view ([V,N], e.g. the
 * per-camera importance I_k(s) that SH compaction weighs its rows with, Sec. 4.4).
 * Every (tile, splat) partial sum is multiplied by o_weight before it is added:
 * 1 keeps the raw sums; 1/P (P = pixels of the view) makes importance the
 * paper's I_k(s); 1/(V P) its camera average I_k; 1/(3 V P) makes scores_se the
 * paper's dMSE_k (Sec. 4.2, the average over V cameras, P pixels, 3 channels).
 * Outputs are ACCUMULATED (+=); zero them first. A weight must be finite and > 0.
 * ------------------------------------------------------------------------- */
typedef struct potr_outputs {
    float* scores;
    int64_t scores_stride;
    float scores_weight;
    float* scores_se;
    int64_t se_stride;
    float se_weight;
    float* importance;
    int64_t importance_stride;
    float importance_weight;
    int32_t fixed_point;   /* 1: the three arrays are int64 fixed-point sums (below) */
} potr_outputs;

/* potr_fixed_to_float -- out[i] = acc[i] * 2^-32 for n elements (device arrays).
 * For callers that need run-to-run reproducible sums: with
 * potr_outputs.fixed_point = 1, scores, scores_se and importance point to int64
 * arrays in units of 2^-32 (strides in elements). Each wave's sum of a (tile,
 * splat) is rounded to that grid, and the sums over waves, tiles and views are
 * integer adds, which commute: the result does not depend on the order the
 * hardware takes them in, so repeated runs give the same bits. The rounding
 * costs at most 2^-33 per wave sum; totals must stay below 2^31 in magnitude.
 * The fused pass in this mode keeps 8-byte per-entry sums in LDS. */
POTR_API potr_status potr_fixed_to_float(const int64_t* acc, int64_t n, float* out, void* stream);

/* potr_render_score_out -- potr_render_score with its reductions described by
 * `out` (host struct): per-view arrays and weights as above. image may be NULL;
 * at least one output (image included) must be requested. */
POTR_API potr_status potr_render_score_out(int64_t N, int32_t V, const potr_camera* cams, const potr_config* cfg,
                                           const potr_proj* proj, const uint32_t* sorted_ids,
                                           const int32_t* tile_ranges, float* image, const float* target,
                                           const potr_outputs* out, void* stream);

/* ---------------------------------------------------------------------------
 * Batched scoring of many scenes and views of uneven sizes (the paper scores
 * every training view of a model per pruning iteration, Sec. 4.3).
 *
 * A job is one scene and a run of its views (one image size per job). The
 * batch runs project -> bin -> sort per job and then ONE persistent launch of
 * the fused render + removal pass whose workgroups pull (view, tile) items of
 * all jobs from a device counter until none is left. All of it can be
 * recorded into one HIP graph and replayed.
 *
 * potr_batch_create: validates, copies the job table (cameras included) and
 *   counts each job's tile pairs by projecting it once: this call synchronises
 *   `stream` and uses temporary device memory. Pair capacity per job =
 *   count * (1 + margin) + 1024.
 * potr_batch_workspace_size / potr_batch_bind: the caller supplies one device
 *   workspace; bind uploads the job table into it (synchronises). The render's
 *   queue holds the jobs' items by decreasing mean counted pairs per tile, so
 *   the cheapest tiles are the last ones drawn.
 * potr_batch_pairs: counted pairs and capacities per job (host arrays [n_jobs]).
 * potr_batch_run: enqueues the whole batch; no allocation, no host sync, safe to
 *   capture. Jobs run in up to four lanes (own scratch in the workspace, own
 *   default-priority stream created with the batch), forked from `stream` after
 *   the work already on it and joined back before the render launch. Scores
 *   accumulate (+=) into each job's buffers; a job with a fine-tuning step runs
 *   it in its lane right after its tile lists (forward composite, loss gradient,
 *   blend and projection backward), so the step's gradients are in the same
 *   run (and the same graph) as the scores.
 * potr_batch_render: enqueues only the persistent render + removal launch over
 *   the tile lists the last run (or replay) left in the workspace; scores
 *   accumulate (+=) again. With the lists unchanged it adds the same sums (up to
 *   float addition order): a way to time or repeat the dominant launch alone.
 * potr_batch_capture / potr_batch_replay: record potr_batch_run into a graph on
 *   `stream` (not the null stream) / launch it.
 * potr_batch_overflow: after a run, the number of jobs whose pairs exceeded
 *   their capacity (synchronises). Such a job contributes nothing; re-create the
 *   batch with a larger margin.
 * Calls that share a batch must not overlap.
 * ------------------------------------------------------------------------- */
typedef struct potr_job {
    int64_t N;
    const float *means, *scales, *quats, *opac, *sh;  /* device, as for potr_project */
    int32_t V;
    const potr_camera* cams;                          /* host [V], copied at create */
    potr_outputs out;                                 /* device outputs of this job's views, as for
                                                         potr_render_score_out */
    const float* target;                              /* device [V,H,W,3], needed with out.scores_se */
    /* Optional fine-tuning step (Sec. 4.6): with grad_target [V,H,W,3] (device)
       the batch also composites the job's views, forms the gradient of the
       loss grad_weight * sum over pixels and channels of |image - grad_target|
       (sign(0) = 0) and runs the backward, ADDING the gradients into d_means
       [N,3], d_scales [N,3], d_quats [N,4], d_opac [N] and d_sh [N,16,3]
       (device, all five needed). Jobs that add into the same gradient arrays
       run in one lane, one after another. A job needs score outputs, a
       fine-tuning step, or both. */
    const float* grad_target;
    float grad_weight;
    float *d_means, *d_scales, *d_quats, *d_opac, *d_sh;
} potr_job;

typedef struct potr_batch_s* potr_batch;

POTR_API potr_status potr_batch_create(const potr_job* jobs, int32_t n_jobs, const potr_config* cfg, float margin,
                                       potr_batch* out, void* stream);
POTR_API potr_status potr_batch_workspace_size(potr_batch b, size_t* bytes);
POTR_API potr_status potr_batch_pairs(potr_batch b, int64_t* counted, int64_t* capacity);
POTR_API potr_status potr_batch_bind(potr_batch b, void* ws, size_t ws_bytes, void* stream);
POTR_API potr_status potr_batch_run(potr_batch b, void* stream);
POTR_API potr_status potr_batch_render(potr_batch b, void* stream);
POTR_API potr_status potr_batch_capture(potr_batch b, void* stream);
POTR_API potr_status potr_batch_replay(potr_batch b, void* stream);
POTR_API potr_status potr_batch_overflow(potr_batch b, int32_t* n_overflowed, void* stream);
POTR_API potr_status potr_batch_destroy(potr_batch b);

/* ---------------------------------------------------------------------------
 * Pruning controller (Sec. 4.3), one iteration on the device.
 *
 * potr_prune_select: which splats one iteration removes, from every splat's
 *   dMSE_k and importance I_k (Sec. 4.1, 4.2; normalised as the paper defines
 *   them, e.g. by potr_render_score_out's weights). Candidates are the splats with
 *   dMSE_k < dmse_max; the budget is B = (sum of the candidates' I_k) / remaining,
 *   `remaining` the iterations still to run, this one included; candidates are
 *   taken in ascending order of m(dMSE_k / dmse_max), m(x) = x for x >= 0 and
 *   (sqrt(1 - 2 a x) - 1) / a for x < 0, ties by index, until B <= the importance
 *   taken (that splat included). Nothing is removed when B = 0; a splat with
 *   dMSE_k >= dmse_max is never removed.
 *   Exact rules: x and m(x) are correctly rounded FP64 operations in that order;
 *   each I_k is rounded to a multiple of 2^-52 and the budget is compared in
 *   those integers (first prefix reaching ceil(total / remaining)), so no
 *   summation order moves the cut.
 *   dmse, importance [N] FP32 (device); importance must lie in [0, 1] with a
 *     candidate sum of at most 2 (an image fraction), else *n_removed = -1 and
 *     nothing is removed
 *   dmse_max > 0 (the paper's dMSE_MAX), a > 0 (the paper uses 10), remaining >= 1
 *   ws     workspace of potr_prune_workspace_size(N) bytes
 *   remove [N] uint8 out: 1 for a removed splat
 *   n_removed (device) int64 out: how many (or -1, see above)
 * potr_prune_compact: the survivors (remove[k] == 0) in index order: each splat
 *   array of potr_project's layout is copied to its *_out array (N_kept rows),
 *   ids_out gets ids[k] (or k when ids is NULL), *n_kept (device int64) the
 *   count. Outputs must not overlap the inputs; quats and sh 16-byte aligned.
 * Both only enqueue work (no allocation, no host synchronisation).
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_prune_workspace_size(int64_t N, size_t* bytes);
POTR_API potr_status potr_prune_select(int64_t N, const float* dmse, const float* importance, double dmse_max,
                                       int32_t remaining, double a, void* ws, size_t ws_bytes, uint8_t* remove,
                                       int64_t* n_removed, void* stream);
POTR_API potr_status potr_prune_compact(int64_t N, const uint8_t* remove, const float* means, const float* scales,
                                        const float* quats, const float* opac, const float* sh, const int32_t* ids,
                                        void* ws, size_t ws_bytes, float* means_out, float* scales_out,
                                        float* quats_out, float* opac_out, float* sh_out, int32_t* ids_out,
                                        int64_t* n_kept, void* stream);

/* ---------------------------------------------------------------------------
 * potr_sh_compact -- spherical-harmonics energy compaction (Sec. 4.4): new
 * lighting coefficients per splat that keep the colours its training cameras
 * see, at lower energy. Per splat and colour channel (in YCoCg: Y = R/4 + G/2 +
 * B/4, Co = R/2 - B/2, Cg = -R/4 + G/2 - B/4), with Y the SH basis at the unit
 * directions from each camera centre to the splat (rows weighted by the
 * camera's importance over the splat's largest) and C = Y L the colours (the raw
 * SH sum, before the renderer's +1/2 and clamp):
 *   - an AC column is dropped (coefficient 0) when |cosine| with a kept column
 *     before it exceeds alpha (the DC is always kept; a zero column is dropped);
 *   - ridge regression L' = (Y^T Y + Gamma^T Gamma)^-1 Y^T C over the kept
 *     columns, Gamma = sqrt(lam_c) diag(0, 1, .., 1), lam_Y = lam,
 *     lam_Co = lam_Cg = 3 lam;
 *   - AC coefficients with |L'_i| < tau are forced to 0 and the ridge problem is
 *     solved again over the rest;
 *   - back to RGB (R = Y + Co - Cg, G = Y + Cg, B = Y - Co - Cg).
 * A splat no camera sees keeps its DC and gets AC 0; coefficients beyond
 * sh_degree are set to 0. The paper's hyperparameters at quality q: lam = 10^-q,
 * alpha = sigmoid(3 q); tau = 1/(2 (1 + 100 q)) is half the SH quantiser's step.
 *   cams (host) [V]; importance [V, stride] FP32 (device): the per-camera
 *     importance I_k(s) (e.g. from potr_render_score_out with a per-view
 *     stride); means [N,3], sh [N,16,3] as for potr_project
 *   ws  workspace of potr_sh_compact_workspace_size(N, V) bytes (per splat 137
 *       doubles, its Gram matrix and largest importance, and a 4-byte slot of
 *       the list of splats some camera sees)
 *   sh_out [N,16,3] FP32 out (must not overlap sh)
 * Arithmetic: FP64 (the Gram matrices on the FP64 matrix cores).
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_sh_compact_workspace_size(int64_t N, int32_t V, size_t* bytes);
POTR_API potr_status potr_sh_compact(int64_t N, int32_t V, const potr_camera* cams, int32_t sh_degree,
                                     const float* means, const float* sh, const float* importance,
                                     int64_t importance_stride, double lam, double alpha, double tau, void* ws,
                                     size_t ws_bytes, float* sh_out, void* stream);

/* ---------------------------------------------------------------------------
 * potr_prune_select_noalloc -- for callers that cannot allocate device memory
 * (code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): potr_prune_select without the workspace argument. Its scratch
 * (4 KB: the select's state and histograms, whatever N) is a static device array
 * of the library, one copy per GPU, which each GPU the library runs on keeps
 * until the process ends; the call uses the copy of the current device, so
 * `stream` must belong to the current device. The call clears the scratch
 * itself (with a kernel) before using it. Calls that overlap on one GPU share
 * that scratch and race: order them (one stream, or events between streams).
 * Limits: N <= 2^31 - 1 (larger N is rejected with POTR_EINVAL); other
 * arguments, outputs and errors as potr_prune_select. Allocates nothing and
 * calls no allocating routine; only enqueues work.
 * ------------------------------------------------------------------------- */
POTR_API potr_status potr_prune_select_noalloc(int64_t N, const float* dmse, const float* importance,
                                               double dmse_max, int32_t remaining, double a, uint8_t* remove,
                                               int64_t* n_removed, void* stream);

/* ---------------------------------------------------------------------------
 * Codec (paper Sec. 4.5; hyperparameters of the Sec. 5.1 table). Encoder: the
 * attributes are quantised uniformly, x_hat = floor(1/2 + x SF) with one scale
 * factor per attribute (activated scale, unit quaternion x, y, z with w >= 0,
 * activated opacity, every SH coefficient; DC coefficients as differences to
 * the previous splat); positions go to the centre of an octree leaf, a node
 * being split while it holds more than one splat or its one splat misses
 * |mu - centre| < max(gamma, beta * distance to the nearest training camera
 * eye); the octree is written depth first, one occupancy byte per node (bit
 * c = x | y << 1 | z << 2 for each child octant, 0 for a leaf), then the
 * attributes in that leaf order, one property after another; zstd last.
 * Decoder: the reverse, opacity dequantised a quarter step up, (x_hat + 1/4) / SF.
 *
 * Where the paper leaves the format open: the root is the cube at the per-axis
 * minimum of the positions with side (largest extent) * (1 + 2^-20); positions
 * are placed on a 2^max_depth grid per axis and nodes at max_depth are leaves
 * whatever they hold (their splat counts are stored, u32 each); the precision
 * test compares squares in FP64. Layout, little-endian: a 104-byte header
 * (magic "POTR", version 1, N, max_depth, sh_degree, lo[3], size, the four
 * scale factors, node and cap-leaf counts), the node bytes, the cap-leaf
 * counts, then 7 + 3 (sh_degree + 1)^2 int32 streams of N values: opacity,
 * scale x y z, rotation x y z, SH coefficient j channel r g b.
 *
 * potr_codec_encode (device inputs as for potr_project: means [N,3], scales
 *   [N,3], quats [N,4] (w,x,y,z), opacities [N], sh [N,16,3] of which the first
 *   (sh_degree+1)^2 coefficients are coded; cams: host array of the training
 *   cameras, whose eyes set the precision bound): writes the uncompressed
 *   bitstream into the host buffer raw (raw_cap bytes, at most
 *   potr_codec_max_bytes) and its size into *raw_bytes (also when the buffer is
 *   too small: POTR_ECAPACITY). leaf_order (device [N], optional): the input
 *   index of each coded splat. ws: potr_codec_workspace_size bytes of device
 *   memory. Synchronises `stream` (to size the octree bytes, then to copy
 *   the bitstream out).
 *   POTR_EINVAL for non-finite positions or a quantised value outside int32.
 * potr_codec_compress / potr_codec_decompress: zstd at `level` through the
 *   system's libzstd.so.1 (POTR_EUNSUPPORTED when it cannot be loaded).
 * potr_codec_info / potr_codec_decode: N and sh_degree of a bitstream, and the
 *   decoded model into host arrays (layouts as above; the splats in leaf
 *   order, SH coefficients past sh_degree zero). POTR_EINVAL for a stream that
 *   does not parse.
 * ------------------------------------------------------------------------- */
typedef struct potr_codec_params {
    double beta, gamma;                          /* precision test */
    double sf_scale, sf_rot, sf_opac, sf_sh;     /* quantisation scale factors */
    int32_t max_depth;                           /* octree depth cap, 1..21 */
    int32_t reserved;
} potr_codec_params;

POTR_API potr_status potr_codec_workspace_size(int64_t N, int32_t sh_degree, int32_t n_cams, size_t* bytes);
POTR_API potr_status potr_codec_max_bytes(int64_t N, int32_t sh_degree, int32_t max_depth, size_t* bytes);
POTR_API potr_status potr_codec_encode(int64_t N, const float* means, const float* scales, const float* quats,
                                       const float* opacities, const float* sh, int32_t sh_degree,
                                       const potr_camera* cams, int32_t n_cams, const potr_codec_params* prm,
                                       void* ws, size_t ws_bytes, uint8_t* raw, size_t raw_cap, size_t* raw_bytes,
                                       uint32_t* leaf_order, void* stream);
POTR_API potr_status potr_codec_compress_bound(size_t raw_bytes, size_t* bytes);
POTR_API potr_status potr_codec_compress(const uint8_t* raw, size_t raw_bytes, int32_t level, uint8_t* out,
                                         size_t out_cap, size_t* out_bytes);
POTR_API potr_status potr_codec_decompressed_size(const uint8_t* comp, size_t comp_bytes, size_t* raw_bytes);
POTR_API potr_status potr_codec_decompress(const uint8_t* comp, size_t comp_bytes, uint8_t* raw, size_t raw_cap,
                                           size_t* raw_bytes);
POTR_API potr_status potr_codec_info(const uint8_t* raw, size_t raw_bytes, int64_t* N, int32_t* sh_degree);
POTR_API potr_status potr_codec_decode(const uint8_t* raw, size_t raw_bytes, float* means, float* scales,
                                       float* quats, float* opacities, float* sh);

/* potr_autotune: times every tile shape (16x16, 8x8, 32x8) with every LDS batch
 * (64, 128, 320, 512) on the given jobs (`reps` timed runs each, after one
 * warm-up) and writes the fastest tile_w, tile_h, lds_batch into *inout. Uses
 * temporary device memory and scratch scores, and leaves fine-tuning steps out
 * (the jobs' outputs and gradients are untouched);
 * synchronises. A shape at which some job's pairs exceed one call's limit
 * (2^31 - 1) is skipped; POTR_EINVAL when no candidate fits. Optional:
 * best_ms, and the tried configs with their times (arrays of at least 12) and
 * their count. */
POTR_API potr_status potr_autotune(const potr_job* jobs, int32_t n_jobs, potr_config* inout, int32_t reps,
                                   double* best_ms, potr_config* tried, double* tried_ms, int32_t* n_tried,
                                   void* stream);

#ifdef __cplusplus
}
#endif
#endif /* POTR_H */
