// Per-(pixel, splat) arithmetic shared by the blend, score and backward
// kernels. Every operation is an explicit round-to-nearest intrinsic, so the
// compiler cannot contract or reorder it differently in different kernels: the
// three passes take the same visibility decisions and accumulate the same
// transmittance and partial colour, bit for bit.
#pragma once

#include <hip/hip_runtime.h>

namespace potr {

// exp(-q/2) = exp2(s q) with s = -log2(e)/2 (halving the FP32 log2(e) is exact).
// Staged records carry the conic pre-multiplied by s, so a sweep forms the
// exponent e = s q of the quadratic form directly.
constexpr float kExpScale = -0x1.715476p-1f;

// Staged record from the first two 16-byte words of a potr_proj
// (r0 = mean2d.x, mean2d.y, conic.a, conic.b; r1 = conic.c, opacity, r, g):
//   a = (mean2d.x, mean2d.y, opacity, s 2 conic.b), b = (s conic.a, s conic.c, r, g)
// (blue is staged separately). Each scaled value is one FP32 rounding.
__device__ inline void make_rec(const float4& r0, const float4& r1, float4& a, float4& b) {
    a = make_float4(r0.x, r0.y, r1.y, __fmul_rn(2.f * r0.w, kExpScale));
    b = make_float4(__fmul_rn(r0.z, kExpScale), __fmul_rn(r1.x, kExpScale), r1.z, r1.w);
}

// The q <= q_max test as a test on the exponent: e >= emin
__device__ inline float exp_floor(float qmax) { return __fmul_rn(qmax, kExpScale); }

struct Gauss {
    float dx, dy;   // centre minus pixel centre
    float e;        // s (a dx^2 + 2 b dx dy + c dy^2) = s q
    float G;        // exp2(e) = exp(-q/2)
    float al0;      // o G (before the alpha_max clamp)
};

__device__ inline Gauss eval_gauss(const float4& a, const float4& b, float fx, float fy) {
    Gauss r;
    r.dx = __fsub_rn(a.x, fx);
    r.dy = __fsub_rn(a.y, fy);
    // e = dx (sa dx + s2b dy) + (sc dy) dy
    const float t = __fmaf_rn(b.x, r.dx, __fmul_rn(a.w, r.dy));
    const float u = __fmul_rn(b.y, r.dy);
    r.e = __fmaf_rn(r.dx, t, __fmul_rn(u, r.dy));
    r.G = __builtin_amdgcn_exp2f(r.e);
    r.al0 = __fmul_rn(a.z, r.G);
    return r;
}

// alpha where the splat counts at this pixel (q <= q_max, o G >= alpha_min), else 0
__device__ inline float alpha_of(const Gauss& g, float emin, float amin, float amax) {
    return (g.e >= emin && g.al0 >= amin) ? fminf(amax, g.al0) : 0.f;
}

// the same, and 0 where `live` is false (one select for all three tests)
__device__ inline float alpha_if(const Gauss& g, float emin, float amin, float amax, bool live) {
    return (live && g.e >= emin && g.al0 >= amin) ? fminf(amax, g.al0) : 0.f;
}

__device__ inline float next_T(float T, float al) { return __fmul_rn(T, __fsub_rn(1.f, al)); }

__device__ inline float add_weighted(float P, float w, float c) { return __fmaf_rn(w, c, P); }

// Tile rows [r0, r1] (relative to the tile's first row, packed r0 | r1 << 8;
// r0 > r1 when none) that a staged record can reach: pixel centres within the
// vertical extent of the ellipse q <= q_max, |dy| <= sqrt(q_max a / (a c - b^2)),
// widened by 2^-10 relative + 1/64 px so that no FP32 evaluation inside the
// rows it excludes could pass the visibility test. Used to skip whole waves.
__device__ inline uint32_t reach_rows(const float4& a, const float4& b, float qmax, int tile_y0, int TH) {
    // FP64: the products of FP32 values are exact, so det has one rounding even
    // for very elongated ellipses. The staged conic is s times the conic
    // (s < 0): its det is s^2 times the conic's, so (A s) / det here is the
    // conic's a / det.
    const double A = b.x, B = 0.5 * (double)a.w, Cc = b.y;
    const double det = A * Cc - B * B;
    int r0 = 0, r1 = TH - 1;
    if (det > 0.0) {
        const double ry = sqrt((double)qmax * A * (double)kExpScale / det) * (1.0 + 1.0 / 1024.0) + 1.0 / 64.0;
        if (ry == ry && ry < 1e8) {
            // rows j with |j + 0.5 - my| <= ry
            const double lo = ceil((double)a.y - ry - 0.5) - (double)tile_y0;
            const double hi = floor((double)a.y + ry - 0.5) - (double)tile_y0;
            r0 = lo < 0.0 ? 0 : (lo > (double)(TH - 1) ? TH : (int)lo);
            r1 = hi > (double)(TH - 1) ? TH - 1 : (hi < 0.0 ? -1 : (int)hi);
        }
    }
    if (r0 > r1) return 0xffu;          // r0 = 255, r1 = 0: reaches no row
    return (uint32_t)r0 | ((uint32_t)r1 << 8);
}

__device__ inline bool rows_overlap(uint32_t rr, int row_lo, int row_hi) {
    const int r0 = (int)(rr & 0xffu), r1 = (int)(rr >> 8);
    return r0 <= row_hi && r1 >= row_lo;
}

// 1 / (1 - alpha) with the hardware reciprocal (1 ulp), 1 - alpha >= 1 - alpha_max
__device__ inline float inv_keep(float al) { return __builtin_amdgcn_rcpf(__fsub_rn(1.f, al)); }

// Colour still to come behind a splat: R = Q - P with Q = P_K + T_final bg and
// P the partial colour through the splat; each blended splat takes w c off it.
__device__ inline float sub_weighted(float R, float w, float c) { return __fmaf_rn(-w, c, R); }

// Removal effect of one splat on one channel of one pixel, -w c + alpha/(1-alpha) R
// with R = Q - P through the splat. Since R_prev = R + w c is the value before the
// splat, it equals R / (1 - alpha) - R_prev: one FMA per channel.
__device__ inline float removal_delta(float inv, float R, float R_prev) { return __fmaf_rn(inv, R, -R_prev); }

// Per-wave list of the staged entries [0, cnt) whose reachable tile rows
// (rows[j * STRIDE] for entry j) meet the wave's rows [row_lo, row_hi], in
// increasing order; returns its length.
// The list is written and read by the same wave only (LDS operations of one
// wave complete in order).
template <int STRIDE = 1>
__device__ inline int wave_list(const uint32_t* rows, int cnt, int row_lo, int row_hi, uint16_t* list) {
    const int lane = threadIdx.x & 63;
    const uint64_t below = (1ull << lane) - 1ull;
    int n = 0;
    for (int c0 = 0; c0 < cnt; c0 += 64) {
        const int j = c0 + lane;
        const bool ok = j < cnt && rows_overlap(rows[j * STRIDE], row_lo, row_hi);
        const uint64_t m = __ballot(ok);
        if (ok) list[n + __popcll(m & below)] = (uint16_t)j;
        n += __popcll(m);
    }
    __builtin_amdgcn_wave_barrier();
    return n;
}

}  // namespace potr
