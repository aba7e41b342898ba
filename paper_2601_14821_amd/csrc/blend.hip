// Front-to-back alpha compositing (paper Sec. 3) and the removal pass (Sec. 4.2).
//
// One workgroup per (tile, view), one thread per pixel: 16x16 and 32x8 tiles are
// four wave64s, 8x8 is one. The tile's depth-sorted records are staged through
// LDS in batches of cfg.lds_batch; every lane of a wave then reads the same LDS
// record (a broadcast, no bank conflicts) and evaluates it for its own pixel.
//
// potr_score walks each pixel's visited prefix again, front to back, and forms
//   PD_k = -c_k w_k + alpha_k/(1-alpha_k) (S_k + T_final bg),
//   w_k = T_k alpha_k,  S_k = P_K - P_{k+1},
// which equals the paper's P_{i_k} - P_{i_k+1}/(1-alpha) + alpha/(1-alpha) P_K
// (with the background term added) since P_{k+1} = P_k + w_k c_k. Per splat the
// pixel values are summed across the wave with cross-lane shuffles, across the
// waves of the tile through LDS, and then added to the per-splat output with one
// device atomic per (tile, splat) that has a nonzero sum.
#include "common.h"
#include "dpp.h"
#include "raster_eval.h"

namespace potr {
namespace {

constexpr int kMaxBatch = 512;

template <int NT, int TH>
__device__ inline void stage_batch(const potr_proj* __restrict__ pv, const uint32_t* __restrict__ ids, int base,
                                   int cnt, float4* s_a, float4* s_b, float* s_c, uint32_t* s_id, uint32_t* s_rows,
                                   float qmax, int tile_y0) {
    for (int j = threadIdx.x; j < cnt; j += NT) {
        const uint32_t id = ids[base + j];
        const float4* src = reinterpret_cast<const float4*>(pv + id);
        const float4 r0 = src[0];   // mean2d.x, mean2d.y, conic.a, conic.b
        const float4 r1 = src[1];   // conic.c, opacity, r, g
        const float4 r2 = src[2];   // b, depth, rect
        float4 a, b;
        make_rec(r0, r1, a, b);
        s_a[j] = a;
        s_b[j] = b;
        s_c[j] = r2.x;
        s_rows[j] = reach_rows(a, b, qmax, tile_y0, TH);
        if (s_id) s_id[j] = id;
    }
}

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_blend(int64_t N, int32_t W, int32_t H, int32_t tiles_x,
                                                   int32_t tiles_per_view, potr_config cfg,
                                                   const potr_proj* __restrict__ proj,
                                                   const uint32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges, float* __restrict__ image,
                                                   float* __restrict__ p_final, float* __restrict__ t_final,
                                                   int32_t* __restrict__ n_walk, int32_t* __restrict__ n_blend) {
    constexpr int NT = TW * TH;
    // LDS sized by the run's batch (blend_lds_bytes): records, reachable rows, per-wave lists
    extern __shared__ __align__(16) char smem[];
    const int B = cfg.lds_batch;
    float4* const s_a = reinterpret_cast<float4*>(smem);
    float4* const s_b = s_a + B;
    float* const s_c = reinterpret_cast<float*>(s_b + B);
    uint32_t* const s_rows = reinterpret_cast<uint32_t*>(s_c + B);
    uint16_t* const s_list = reinterpret_cast<uint16_t*>(s_rows + B);   // [NW][B]
    const int tile = blockIdx.x, v = blockIdx.y;
    const int wid = threadIdx.x >> 6;
    const int row_lo = __builtin_amdgcn_readfirstlane((wid * 64) / TW);
    const int row_hi = __builtin_amdgcn_readfirstlane((wid * 64 + 63) / TW);
    const int tile_y0 = (tile / tiles_x) * TH;
    const int px = (tile % tiles_x) * TW + (int)(threadIdx.x % TW);
    const int py = tile_y0 + (int)(threadIdx.x / TW);
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int64_t tg = (int64_t)v * tiles_per_view + tile;
    const int beg = ranges[2 * tg], end = ranges[2 * tg + 1];
    const potr_proj* pv = proj + (int64_t)v * N;
    const float qmax = cfg.q_max, amin = cfg.alpha_min, amax = cfg.alpha_max, tmin = cfg.t_min;
    const float emin = exp_floor(qmax);

    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
    bool done = !inside;
    int walk = 0, blended = 0;
    for (int base = beg; base < end; base += B) {
        if (__syncthreads_count(!done) == 0) break;
        const int cnt = min(B, end - base);
        stage_batch<NT, TH>(pv, ids, base, cnt, s_a, s_b, s_c, nullptr, s_rows, qmax, tile_y0);
        __syncthreads();
        // this wave's entries (those reaching its rows), each step branch-free: a
        // finished lane takes alpha = 0, which leaves T and the colour unchanged
        uint16_t* const L = s_list + wid * B;
        const int nl = wave_list(s_rows, cnt, row_lo, row_hi, L);
        if (__ballot(!done) == 0) continue;
        for (int i = 0; i < nl; i += 4) {
            const uint2 q = *reinterpret_cast<const uint2*>(L + i);
            const uint32_t qx = __builtin_amdgcn_readfirstlane(q.x), qy = __builtin_amdgcn_readfirstlane(q.y);
            const int js[4] = {(int)(qx & 0xffffu), (int)(qx >> 16), (int)(qy & 0xffffu), (int)(qy >> 16)};
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i + u >= nl) break;
                const int j = js[u];
                const float4 b = s_b[j];
                const float a0 = alpha_of(eval_gauss(s_a[j], b, fx, fy), emin, amin, amax);
                const float al = done ? 0.f : a0;
                float Tn = next_T(T, al);
                const bool stop = Tn < tmin;       // T >= tmin before, so only when al > 0
                float w = __fmul_rn(T, al);
                // a lane stops once per tile: only entries where some lane of the
                // wave stops take the selects (the lane keeps T and adds nothing)
                if (__ballot(stop) != 0) {
                    w = stop ? 0.f : w;
                    Tn = stop ? T : Tn;
                    walk = stop ? base - beg + j : walk;
                    done = done || stop;
                }
                cr = add_weighted(cr, w, b.z);
                cg = add_weighted(cg, w, b.w);
                cb = add_weighted(cb, w, s_c[j]);
                T = Tn;
                blended += (al != 0.f && !stop) ? 1 : 0;
            }
            if (__ballot(!done) == 0) break;
        }
    }
    if (!inside) return;
    if (!done) walk = end - beg;
    const int64_t pix = ((int64_t)v * H + py) * W + px;
    image[3 * pix] = __fadd_rn(cr, __fmul_rn(T, cfg.bg[0]));
    image[3 * pix + 1] = __fadd_rn(cg, __fmul_rn(T, cfg.bg[1]));
    image[3 * pix + 2] = __fadd_rn(cb, __fmul_rn(T, cfg.bg[2]));
    if (p_final) {
        p_final[3 * pix] = cr;
        p_final[3 * pix + 1] = cg;
        p_final[3 * pix + 2] = cb;
    }
    if (t_final) t_final[pix] = T;
    if (n_walk) n_walk[pix] = walk;
    if (n_blend) n_blend[pix] = blended;
}

template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) void k_score(int64_t N, int32_t W, int32_t H, int32_t tiles_x,
                                                   int32_t tiles_per_view, potr_config cfg,
                                                   const potr_proj* __restrict__ proj,
                                                   const uint32_t* __restrict__ ids,
                                                   const int32_t* __restrict__ ranges,
                                                   const float* __restrict__ p_final,
                                                   const float* __restrict__ t_final,
                                                   const int32_t* __restrict__ n_walk,
                                                   const float* __restrict__ target, float* __restrict__ scores,
                                                   float* __restrict__ scores_se, float* __restrict__ importance) {
    constexpr int NT = TW * TH;
    constexpr int NW = (NT + 63) / 64;
    __shared__ float4 s_a[kMaxBatch];
    __shared__ float4 s_b[kMaxBatch];
    __shared__ float s_c[kMaxBatch];
    __shared__ uint32_t s_id[kMaxBatch];
    __shared__ uint32_t s_rows[kMaxBatch];
    __shared__ float s_part[3][NW][kMaxBatch];
    __shared__ int s_wmax;
    const int tile = blockIdx.x, v = blockIdx.y;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int row_lo = __builtin_amdgcn_readfirstlane((wid * 64) / TW);
    const int row_hi = __builtin_amdgcn_readfirstlane((wid * 64 + 63) / TW);
    const int tile_y0 = (tile / tiles_x) * TH;
    const int px = (tile % tiles_x) * TW + (int)(threadIdx.x % TW);
    const int py = tile_y0 + (int)(threadIdx.x / TW);
    const bool inside = px < W && py < H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int64_t tg = (int64_t)v * tiles_per_view + tile;
    const int beg = ranges[2 * tg];
    const potr_proj* pv = proj + (int64_t)v * N;
    const int B = cfg.lds_batch;
    const float qmax = cfg.q_max, amin = cfg.alpha_min, amax = cfg.alpha_max;
    const float emin = exp_floor(qmax);
    const bool want_l1 = scores != nullptr, want_se = scores_se != nullptr, want_im = importance != nullptr;

    int walk = 0;
    float Qr = 0.f, Qg = 0.f, Qb = 0.f, er = 0.f, eg = 0.f, eb = 0.f;   // Q = P_K + T_final bg
    const int64_t pix = ((int64_t)v * H + py) * W + px;
    if (inside) {
        walk = n_walk[pix];
        const float TF = t_final[pix];
        Qr = __fadd_rn(p_final[3 * pix], __fmul_rn(TF, cfg.bg[0]));
        Qg = __fadd_rn(p_final[3 * pix + 1], __fmul_rn(TF, cfg.bg[1]));
        Qb = __fadd_rn(p_final[3 * pix + 2], __fmul_rn(TF, cfg.bg[2]));
        if (want_se) {   // c - c_t
            er = Qr - target[3 * pix];
            eg = Qg - target[3 * pix + 1];
            eb = Qb - target[3 * pix + 2];
        }
    }
    if (threadIdx.x == 0) s_wmax = 0;
    __syncthreads();
    atomicMax(&s_wmax, walk);
    __syncthreads();
    const int wmax = s_wmax;

    float T = 1.f, Rr = Qr, Rg = Qg, Rb = Qb;   // Q - P: colour still to come
    for (int base = 0; base < wmax; base += B) {
        const int cnt = min(B, wmax - base);
        stage_batch<NT, TH>(pv, ids, beg + base, cnt, s_a, s_b, s_c, s_id, s_rows, qmax, tile_y0);
        __syncthreads();
        for (int j = 0; j < cnt; ++j) {
            if (!rows_overlap(__builtin_amdgcn_readfirstlane(s_rows[j]), row_lo, row_hi)) {
                if (lane == 0) s_part[0][wid][j] = s_part[1][wid][j] = s_part[2][wid][j] = 0.f;
                continue;
            }
            float l1 = 0.f, se = 0.f, im = 0.f;
            if (base + j < walk) {
                const float4 a = s_a[j];
                const float4 b = s_b[j];
                const float al = alpha_of(eval_gauss(a, b, fx, fy), emin, amin, amax);
                if (al != 0.f) {
                    const float w = __fmul_rn(T, al);
                    const float cr = b.z, cg = b.w, cbl = s_c[j];
                    const float r0 = Rr, r1 = Rg, r2 = Rb;
                    Rr = sub_weighted(Rr, w, cr);
                    Rg = sub_weighted(Rg, w, cg);
                    Rb = sub_weighted(Rb, w, cbl);
                    const float inv = inv_keep(al);
                    const float dr = removal_delta(inv, Rr, r0);
                    const float dg = removal_delta(inv, Rg, r1);
                    const float db = removal_delta(inv, Rb, r2);
                    l1 = fabsf(dr) + fabsf(dg) + fabsf(db);
                    se = dr * dr + dg * dg + db * db + 2.f * (dr * er + dg * eg + db * eb);
                    im = w;
                    T = next_T(T, al);
                }
            }
            if (want_l1) {
                const float s = __ballot(l1 != 0.f) ? wave_sum(l1) : 0.f;
                if (lane == 0) s_part[0][wid][j] = s;
            }
            if (want_se) {
                const float s = __ballot(se != 0.f) ? wave_sum(se) : 0.f;
                if (lane == 0) s_part[1][wid][j] = s;
            }
            if (want_im) {
                const float s = __ballot(im != 0.f) ? wave_sum(im) : 0.f;
                if (lane == 0) s_part[2][wid][j] = s;
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const uint32_t id = s_id[j];
            if (want_l1) {
                float t = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += s_part[0][w][j];
                if (t != 0.f) unsafeAtomicAdd(scores + id, t);
            }
            if (want_se) {
                float t = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += s_part[1][w][j];
                if (t != 0.f) unsafeAtomicAdd(scores_se + id, t);
            }
            if (want_im) {
                float t = 0.f;
#pragma unroll
                for (int w = 0; w < NW; ++w) t += s_part[2][w][j];
                if (t != 0.f) unsafeAtomicAdd(importance + id, t);
            }
        }
        __syncthreads();
    }
}

template <int TW, int TH>
potr_status blend_shape(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg, const potr_proj* proj,
                        const uint32_t* ids, const int32_t* ranges, float* image, float* p_final, float* t_final,
                        int32_t* n_walk, int32_t* n_blend, hipStream_t s) {
    const int txs = tiles_x(c, cfg), tpv = txs * tiles_y(c, cfg);
    constexpr int NW = (TW * TH + 63) / 64;
    const size_t lds = (size_t)cfg.lds_batch * (16 + 16 + 4 + 4 + 2 * NW);
    hipLaunchKernelGGL((k_blend<TW, TH>), dim3(tpv, V), dim3(TW * TH), lds, s, N, c.width, c.height, txs, tpv, cfg,
                       proj, ids, ranges, image, p_final, t_final, n_walk, n_blend);
    return check_launch("k_blend");
}

template <int TW, int TH>
potr_status score_shape(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg, const potr_proj* proj,
                        const uint32_t* ids, const int32_t* ranges, const float* p_final, const float* t_final,
                        const int32_t* n_walk, const float* target, float* scores, float* scores_se,
                        float* importance, hipStream_t s) {
    const int txs = tiles_x(c, cfg), tpv = txs * tiles_y(c, cfg);
    hipLaunchKernelGGL((k_score<TW, TH>), dim3(tpv, V), dim3(TW * TH), 0, s, N, c.width, c.height, txs, tpv, cfg,
                       proj, ids, ranges, p_final, t_final, n_walk, target, scores, scores_se, importance);
    return check_launch("k_score");
}

}  // namespace

potr_status launch_blend(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg, const potr_proj* proj,
                         const uint32_t* ids, const int32_t* ranges, float* image, float* p_final, float* t_final,
                         int32_t* n_walk, int32_t* n_blend, hipStream_t s) {
    if (cfg.tile_w == 16 && cfg.tile_h == 16)
        return blend_shape<16, 16>(N, V, c, cfg, proj, ids, ranges, image, p_final, t_final, n_walk, n_blend, s);
    if (cfg.tile_w == 8 && cfg.tile_h == 8)
        return blend_shape<8, 8>(N, V, c, cfg, proj, ids, ranges, image, p_final, t_final, n_walk, n_blend, s);
    if (cfg.tile_w == 32 && cfg.tile_h == 8)
        return blend_shape<32, 8>(N, V, c, cfg, proj, ids, ranges, image, p_final, t_final, n_walk, n_blend, s);
    return fail(POTR_EUNSUPPORTED, "tile %dx%d not built", cfg.tile_w, cfg.tile_h);
}

potr_status launch_score(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg, const potr_proj* proj,
                         const uint32_t* ids, const int32_t* ranges, const float* p_final, const float* t_final,
                         const int32_t* n_walk, const float* target, float* scores, float* scores_se,
                         float* importance, hipStream_t s) {
    if (cfg.tile_w == 16 && cfg.tile_h == 16)
        return score_shape<16, 16>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, target, scores,
                                   scores_se, importance, s);
    if (cfg.tile_w == 8 && cfg.tile_h == 8)
        return score_shape<8, 8>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, target, scores,
                                 scores_se, importance, s);
    if (cfg.tile_w == 32 && cfg.tile_h == 8)
        return score_shape<32, 8>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, target, scores,
                                  scores_se, importance, s);
    return fail(POTR_EUNSUPPORTED, "tile %dx%d not built", cfg.tile_w, cfg.tile_h);
}

}  // namespace potr
