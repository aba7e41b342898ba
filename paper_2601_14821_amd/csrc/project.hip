// Projection of 3D Gaussians to screen-space records (paper Sec. 3).
//
// One thread per splat; the thread reads the splat's 236 bytes once and loops
// over the views of the launch, so a batch of views costs one parameter read.
// SH coefficients (192 B per splat, contiguous): with one view per launch each
// thread reads its splat's as twelve 16-byte loads issued together (a wave's
// loads cover one contiguous 12 KB span, so every line fetched is used whole
// through the caches; no barrier, no LDS); with several views per launch the
// block's coefficients are first staged in LDS with coalesced 16-byte loads,
// 13 float4 per splat (an odd stride, so a wave's per-splat 16-byte reads hit
// distinct banks), so that the views after the first do not read them again.
// All arithmetic is FP64: CDNA's FP64 vector rate is half its FP32 rate and this
// kernel is bound by HBM (236 B in, 52 B out per splat-view for ~300 flops), so
// FP64 is free here and keeps every stored FP32 value correctly rounded from a
// near-exact result. The depth key is the one exception: a fixed FP32 FMA chain.
#include "common.h"
#include "sh_basis.h"

namespace potr {
namespace {

constexpr int kProjThreads = 128;

// Per-view tangent-plane clamps jclamp * (width / 2) / fx and jclamp * (height / 2) / fy,
// each one FP64 product and one correctly rounded division, formed once per launch.
struct Lims {
    double x[kViewsPerLaunch], y[kViewsPerLaunch];
};

constexpr int kShStride = 13;   // float4 per splat in LDS (12 used)

// DEG: the SH degree in use (0..3), a template argument so that the colour sum
// is fully unrolled with every coefficient and basis value in a register.
// STAGED: SH coefficients staged in LDS (launches of several views).
// KEYS: also write the bin's depth keys, packed rects and per-wave key-range
// partials (BinKeys); every lane of a wave then stays to the end (a lane past
// the last splat repeats the last one and stores nothing), for the wave's max.
template <int DEG, bool STAGED, bool KEYS>
__global__ __launch_bounds__(kProjThreads) void k_project(int64_t N, int32_t v0, int32_t nv, CamBatch cams, Lims lims,
                                                 potr_config cfg, const float* __restrict__ means,
                                                 const float* __restrict__ scales, const float* __restrict__ quats,
                                                 const float* __restrict__ opac, const float* __restrict__ sh,
                                                 potr_proj* __restrict__ proj, int32_t* __restrict__ tiles_touched,
                                                 BinKeys bk) {
    const int64_t i0 = (int64_t)blockIdx.x * kProjThreads;
    const bool live = i0 + threadIdx.x < N;
    const int64_t i = live ? i0 + threadIdx.x : N - 1;
    const float4* sh4;   // this splat's coefficients, 16 bytes at a time
    if constexpr (STAGED) {
        __shared__ float4 s_sh[kProjThreads * kShStride];
        // the float4s holding the 3 (degree + 1)^2 coefficients in use
        const int nb = (int)min((int64_t)kProjThreads, N - i0);
        constexpr int n4 = (3 * (DEG + 1) * (DEG + 1) + 3) / 4;
        const float4* g4 = reinterpret_cast<const float4*>(sh + 48 * i0);
        for (int f = threadIdx.x; f < nb * n4; f += kProjThreads) {
            const int t = f / n4, m = f - t * n4;
            s_sh[t * kShStride + m] = g4[t * 12 + m];
        }
        __syncthreads();
        sh4 = s_sh + (live ? threadIdx.x : i - i0) * kShStride;
    } else {
        sh4 = reinterpret_cast<const float4*>(sh) + 12 * i;
    }
    if (!KEYS && !live) return;

    const float mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const double o = opac[i];
    const float q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const double qn2 = (double)q0 * q0 + (double)q1 * q1 + (double)q2 * q2 + (double)q3 * q3;
    const bool valid = (o >= (double)cfg.alpha_min) && (qn2 > 0.0);

    // 3D covariance Sigma = R(q) diag(s^2) R(q)^T (view independent)
    double S00 = 0, S01 = 0, S02 = 0, S11 = 0, S12 = 0, S22 = 0;
    if (valid) {
        const double inv = 1.0 / sqrt(qn2);
        const double w = q0 * inv, x = q1 * inv, y = q2 * inv, z = q3 * inv;
        const double M[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                             2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                             2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
        const double s0 = (double)scales[3 * i] * scales[3 * i];
        const double s1 = (double)scales[3 * i + 1] * scales[3 * i + 1];
        const double s2 = (double)scales[3 * i + 2] * scales[3 * i + 2];
        S00 = M[0] * M[0] * s0 + M[1] * M[1] * s1 + M[2] * M[2] * s2;
        S01 = M[0] * M[3] * s0 + M[1] * M[4] * s1 + M[2] * M[5] * s2;
        S02 = M[0] * M[6] * s0 + M[1] * M[7] * s1 + M[2] * M[8] * s2;
        S11 = M[3] * M[3] * s0 + M[4] * M[4] * s1 + M[5] * M[5] * s2;
        S12 = M[3] * M[6] * s0 + M[4] * M[7] * s1 + M[5] * M[8] * s2;
        S22 = M[6] * M[6] * s0 + M[7] * M[7] * s1 + M[8] * M[8] * s2;
    }
    constexpr int nsh = (DEG + 1) * (DEG + 1);

    for (int vv = 0; vv < nv; ++vv) {
        const potr_camera& c = cams.c[vv];
        const int64_t out = (int64_t)(v0 + vv) * N + i;
        potr_proj rec;
        rec.mean2d[0] = rec.mean2d[1] = 0.f;
        rec.conic[0] = rec.conic[1] = rec.conic[2] = 0.f;
        rec.opacity = 0.f;
        rec.rgb[0] = rec.rgb[1] = rec.rgb[2] = 0.f;
        rec.rect[0] = rec.rect[1] = rec.rect[2] = rec.rect[3] = 0;
        int32_t ntiles = 0;

        // depth key: t_z + R20 x + R21 y + R22 z, one rounding per fused step
        float z32 = c.t[2];
        z32 = __builtin_fmaf(c.R[6], mx, z32);
        z32 = __builtin_fmaf(c.R[7], my, z32);
        z32 = __builtin_fmaf(c.R[8], mz, z32);
        rec.depth = z32;

        bool ok = valid && (z32 > cfg.near_z);
        if (ok) {
            const double R0 = c.R[0], R1 = c.R[1], R2 = c.R[2], R3 = c.R[3], R4 = c.R[4], R5 = c.R[5],
                         R6 = c.R[6], R7 = c.R[7], R8 = c.R[8];
            const double px = R0 * mx + R1 * my + R2 * mz + (double)c.t[0];
            const double py = R3 * mx + R4 * my + R5 * mz + (double)c.t[1];
            const double pz = R6 * mx + R7 * my + R8 * mz + (double)c.t[2];
            const double fx = c.fx, fy = c.fy;
            const double limx = lims.x[vv], limy = lims.y[vv];
            const double iz = 1.0 / pz;   // one FP64 division; the quotients below are products
            const double tx = fmin(limx, fmax(-limx, px * iz));
            const double ty = fmin(limy, fmax(-limy, py * iz));
            // T = J W (2x3); J = [[fx/z, 0, -fx tx/z], [0, fy/z, -fy ty/z]]
            const double j00 = fx * iz, j02 = -fx * tx * iz, j11 = fy * iz, j12 = -fy * ty * iz;
            const double T00 = j00 * R0 + j02 * R6, T01 = j00 * R1 + j02 * R7, T02 = j00 * R2 + j02 * R8;
            const double T10 = j11 * R3 + j12 * R6, T11 = j11 * R4 + j12 * R7, T12 = j11 * R5 + j12 * R8;
            // cov2d = T Sigma T^T
            const double a0 = T00 * S00 + T01 * S01 + T02 * S02;
            const double a1 = T00 * S01 + T01 * S11 + T02 * S12;
            const double a2 = T00 * S02 + T01 * S12 + T02 * S22;
            const double b0 = T10 * S00 + T11 * S01 + T12 * S02;
            const double b1 = T10 * S01 + T11 * S11 + T12 * S12;
            const double b2 = T10 * S02 + T11 * S12 + T12 * S22;
            const double cxx = a0 * T00 + a1 * T01 + a2 * T02 + (double)cfg.eps2d;
            const double cxy = a0 * T10 + a1 * T11 + a2 * T12;
            const double cyy = b0 * T10 + b1 * T11 + b2 * T12 + (double)cfg.eps2d;
            const double det = cxx * cyy - cxy * cxy;
            const double u = fx * px * iz + (double)c.cx;
            const double v = fy * py * iz + (double)c.cy;
            const double t_cut = fmin((double)cfg.q_max, 2.0 * log(o / (double)cfg.alpha_min));
            const double rx = sqrt(t_cut * cxx) * (1.0 + 1.0 / 1024.0) + 1.0 / 64.0;
            const double ry = sqrt(t_cut * cyy) * (1.0 + 1.0 / 1024.0) + 1.0 / 64.0;
            ok = (det > 0.0) && isfinite(u) && isfinite(v) && isfinite(rx) && isfinite(ry);
            if (ok) {
                rec.mean2d[0] = (float)u;
                rec.mean2d[1] = (float)v;
                const double idet = 1.0 / det;
                rec.conic[0] = (float)(cyy * idet);
                rec.conic[1] = (float)(-cxy * idet);
                rec.conic[2] = (float)(cxx * idet);
                rec.opacity = (float)o;

                // colour along the camera -> centre direction
                const double ex = -(R0 * c.t[0] + R3 * c.t[1] + R6 * c.t[2]);
                const double ey = -(R1 * c.t[0] + R4 * c.t[1] + R7 * c.t[2]);
                const double ez = -(R2 * c.t[0] + R5 * c.t[1] + R8 * c.t[2]);
                double dx = mx - ex, dy = my - ey, dz = mz - ez;
                const double dn = 1.0 / sqrt(dx * dx + dy * dy + dz * dz);
                dx *= dn; dy *= dn; dz *= dn;
                double Y[16];
                sh_basis_d3(dx, dy, dz, DEG, Y);
                double cr = 0.5, cg = 0.5, cb = 0.5;
                // 16-byte loads: four coefficients (r,g,b of k and r of k+1, ...) at a time
                constexpr int n4 = (3 * nsh + 3) / 4;
                float f[4 * n4];
#pragma unroll
                for (int m = 0; m < n4; ++m) {
                    const float4 q = sh4[m];
                    f[4 * m] = q.x;
                    f[4 * m + 1] = q.y;
                    f[4 * m + 2] = q.z;
                    f[4 * m + 3] = q.w;
                }
#pragma unroll
                for (int k = 0; k < nsh; ++k) {
                    cr += (double)f[3 * k] * Y[k];
                    cg += (double)f[3 * k + 1] * Y[k];
                    cb += (double)f[3 * k + 2] * Y[k];
                }
                rec.rgb[0] = (float)fmax(0.0, cr);
                rec.rgb[1] = (float)fmax(0.0, cg);
                rec.rgb[2] = (float)fmax(0.0, cb);

                const double ilo = fmax(ceil(u - rx - 0.5), 0.0), ihi = fmin(floor(u + rx - 0.5), c.width - 1.0);
                const double jlo = fmax(ceil(v - ry - 0.5), 0.0), jhi = fmin(floor(v + ry - 0.5), c.height - 1.0);
                if (ilo <= ihi && jlo <= jhi) {
                    const int x0 = (int)ilo / cfg.tile_w, x1 = (int)ihi / cfg.tile_w + 1;
                    const int y0 = (int)jlo / cfg.tile_h, y1 = (int)jhi / cfg.tile_h + 1;
                    rec.rect[0] = (int16_t)x0; rec.rect[1] = (int16_t)y0;
                    rec.rect[2] = (int16_t)x1; rec.rect[3] = (int16_t)y1;
                    ntiles = (x1 - x0) * (y1 - y0);
                }
            }
        }
        if (live) {
            proj[out] = rec;
            if (tiles_touched) tiles_touched[out] = ntiles;
        }
        if constexpr (KEYS) {
            const uint32_t key = __float_as_uint(rec.depth);
            if (live) {
                bk.keys[out] = key;
                bk.rects[out] = make_uint2((uint32_t)(uint16_t)rec.rect[0] | ((uint32_t)(uint16_t)rec.rect[2] << 16),
                                           (uint32_t)(uint16_t)rec.rect[1] | ((uint32_t)(uint16_t)rec.rect[3] << 16));
            }
            uint32_t hi = key, lo = ~key;   // a repeated last splat leaves the maxima unchanged
#pragma unroll
            for (int m = 32; m >= 1; m >>= 1) {
                hi = max(hi, (uint32_t)__shfl_xor((int)hi, m, 64));
                lo = max(lo, (uint32_t)__shfl_xor((int)lo, m, 64));
            }
            // lane 0 of every wave that holds a splat (a wave wholly past N has none)
            if ((threadIdx.x & 63) == 0 && i0 + threadIdx.x < N)
                bk.part[(int64_t)(v0 + vv) * bk.per_view + (i0 + threadIdx.x) / 64] = make_uint2(hi, lo);
        }
    }
}

}  // namespace

potr_status launch_project(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                           const float* means, const float* scales, const float* quats, const float* opac,
                           const float* sh, potr_proj* proj, int32_t* tiles_touched, hipStream_t s,
                           const BinKeys* keys) {
    if (N == 0) return POTR_OK;
    const dim3 grid((unsigned)ceil_div(N, kProjThreads));
    for (int32_t v0 = 0; v0 < V; v0 += kViewsPerLaunch) {
        const int32_t nv = V - v0 < kViewsPerLaunch ? V - v0 : kViewsPerLaunch;
        CamBatch cb;
        for (int k = 0; k < nv; ++k) cb.c[k] = cams[v0 + k];
        for (int k = nv; k < kViewsPerLaunch; ++k) cb.c[k] = cams[v0];
        Lims lm;
        for (int k = 0; k < kViewsPerLaunch; ++k) {
            lm.x[k] = (double)cfg.jclamp * 0.5 * cb.c[k].width / (double)cb.c[k].fx;
            lm.y[k] = (double)cfg.jclamp * 0.5 * cb.c[k].height / (double)cb.c[k].fy;
        }
        const bool staged = nv > 1;
        const BinKeys bk = keys ? *keys : BinKeys{nullptr, nullptr, nullptr, 0};
        auto go = [&](auto kern) {
            hipLaunchKernelGGL(kern, grid, dim3(kProjThreads), 0, s, N, v0, nv, cb, lm, cfg, means, scales, quats, opac,
                               sh, proj, tiles_touched, bk);
        };
        auto pick = [&](auto k_st_keys, auto k_st, auto k_keys, auto k_plain) {
            if (keys) staged ? go(k_st_keys) : go(k_keys);
            else staged ? go(k_st) : go(k_plain);
        };
        switch (cfg.sh_degree) {
            case 0: pick(k_project<0, true, true>, k_project<0, true, false>, k_project<0, false, true>, k_project<0, false, false>); break;
            case 1: pick(k_project<1, true, true>, k_project<1, true, false>, k_project<1, false, true>, k_project<1, false, false>); break;
            case 2: pick(k_project<2, true, true>, k_project<2, true, false>, k_project<2, false, true>, k_project<2, false, false>); break;
            default: pick(k_project<3, true, true>, k_project<3, true, false>, k_project<3, false, true>, k_project<3, false, false>); break;
        }
        potr_status st = check_launch("k_project");
        if (st != POTR_OK) return st;
    }
    return POTR_OK;
}

}  // namespace potr
