// Per-(pixel, splat) arithmetic shared by the blend, score and backward
// kernels. Every operation is an explicit round-to-nearest intrinsic, so the
// compiler cannot contract or reorder it differently in different kernels: the
// three passes take the same visibility decisions and accumulate the same
// transmittance and partial colour, bit for bit.
#pragma once

#include <hip/hip_runtime.h>

namespace potr {

// Staged record: a = (mean2d.x, mean2d.y, opacity, conic.b), b = (conic.a, conic.c, r, g), c = blue.
struct Gauss {
    float dx, dy;   // centre minus pixel centre
    float q;        // a dx^2 + 2 b dx dy + c dy^2
    float G;        // exp(-q/2)
    float al0;      // o G (before the alpha_max clamp)
};

__device__ inline Gauss eval_gauss(const float4& a, const float4& b, float fx, float fy) {
    Gauss r;
    r.dx = __fsub_rn(a.x, fx);
    r.dy = __fsub_rn(a.y, fy);
    const float ad = __fmul_rn(b.x, r.dx);
    const float bd = __fmul_rn(__fmul_rn(2.f, a.w), r.dx);
    const float cd = __fmul_rn(b.y, r.dy);
    r.q = __fmaf_rn(ad, r.dx, __fmaf_rn(bd, r.dy, __fmul_rn(cd, r.dy)));
    r.G = __expf(__fmul_rn(-0.5f, r.q));
    r.al0 = __fmul_rn(a.z, r.G);
    return r;
}

// alpha where the splat counts at this pixel (q <= q_max, o G >= alpha_min), else 0
__device__ inline float alpha_of(const Gauss& g, float qmax, float amin, float amax) {
    return (g.q <= qmax && g.al0 >= amin) ? fminf(amax, g.al0) : 0.f;
}

__device__ inline float next_T(float T, float al) { return __fmul_rn(T, __fsub_rn(1.f, al)); }

__device__ inline float add_weighted(float P, float w, float c) { return __fmaf_rn(w, c, P); }

}  // namespace potr
