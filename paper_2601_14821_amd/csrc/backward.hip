// Backward of the forward render (the standard 3DGS training pass the paper's
// fine-tuning relies on, Sec. 4.6), for a loss given as dL/dimage.
//
// k_blend_bwd walks every pixel's visited prefix front to back, like the score
// pass, with
//   dC/dc_k     = T_k alpha_k
//   dC/dalpha_k = T_k c_k - (S_k + T_final bg) / (1 - alpha_k),  S_k = P_K - P_{k+1}
// (so the removal effect PD_k = -alpha_k dC/dalpha_k), alpha_k = min(alpha_max,
// o G), G = exp(-q/2), and accumulates per (view, splat) the gradients of the
// 2D record: mean2d (2), conic (3), opacity, rgb (3). Front-to-back recovery of
// T_k avoids dividing by (1 - alpha) as a back-to-front walk would.
//
// k_project_bwd chains those to the splat parameters in FP64, one thread per
// splat, looping over the views of the call.
#include <type_traits>

#include "common.h"
#include "dpp.h"
#include "raster_eval.h"

namespace potr {
namespace {

constexpr int kBwdChunk = 128;   // entries staged per round
constexpr int kG = 9;            // gradient components per (view, splat)

// Compiled for seven waves per SIMD (71 registers, no spills); 8x8 tiles (one
// wave per workgroup, its LDS arrays sized for the tile) take what fits.
template <int TW, int TH>
__global__ __launch_bounds__(TW * TH) __attribute__((amdgpu_waves_per_eu(TW * TH >= 256 ? 7 : 1))) void k_blend_bwd(int64_t N, int32_t W, int32_t H, int32_t tiles_x,
                                                       int32_t tiles_per_view, potr_config cfg,
                                                       const potr_proj* __restrict__ proj,
                                                       const uint32_t* __restrict__ ids,
                                                       const int32_t* __restrict__ ranges,
                                                       const float* __restrict__ p_final,
                                                       const float* __restrict__ t_final,
                                                       const int32_t* __restrict__ n_walk,
                                                       const float* __restrict__ dL_dimage,
                                                       float* __restrict__ grad2d) {
    constexpr int NT = TW * TH;
    constexpr int NW = (NT + 63) / 64;
    __shared__ float4 s_a[kBwdChunk];   // mean2d.x, mean2d.y, opacity, s 2 conic.b (the blend's record)
    __shared__ float4 s_b[kBwdChunk];   // s conic.a, s conic.c, r, g
    __shared__ float4 s_u[kBwdChunk];   // conic.a, conic.b, conic.c (unscaled, for the gradients)
    __shared__ float s_c[kBwdChunk];    // b
    __shared__ uint32_t s_id[kBwdChunk];
    __shared__ uint32_t s_rows[kBwdChunk];
    __shared__ float s_part[kG][kBwdChunk];   // per-entry sums over the waves (LDS float adds)
    __shared__ __align__(8) uint16_t s_list[NW][kBwdChunk];
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
    const float qmax = cfg.q_max, amin = cfg.alpha_min, amax = cfg.alpha_max;
    const float emin = exp_floor(qmax);

    int walk = 0;
    float PKr = 0.f, PKg = 0.f, PKb = 0.f, TF = 0.f, gr = 0.f, gg = 0.f, gb = 0.f;
    if (inside) {
        const int64_t pix = ((int64_t)v * H + py) * W + px;
        walk = n_walk[pix];
        PKr = p_final[3 * pix];
        PKg = p_final[3 * pix + 1];
        PKb = p_final[3 * pix + 2];
        TF = t_final[pix];
        gr = dL_dimage[3 * pix];
        gg = dL_dimage[3 * pix + 1];
        gb = dL_dimage[3 * pix + 2];
    }
    const float Br = TF * cfg.bg[0], Bg = TF * cfg.bg[1], Bb = TF * cfg.bg[2];
    if (threadIdx.x == 0) s_wmax = 0;
    __syncthreads();
    atomicMax(&s_wmax, walk);
    __syncthreads();
    const int wmax = s_wmax;
    // this wave's longest walk: later entries contribute nothing to any of its lanes
    int wave_walk = walk;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) wave_walk = max(wave_walk, __shfl_xor(wave_walk, m, 64));
    wave_walk = __builtin_amdgcn_readfirstlane(wave_walk);

    float T = 1.f, Pr = 0.f, Pg = 0.f, Pb = 0.f;
    for (int base = 0; base < wmax; base += kBwdChunk) {
        const int cnt = min(kBwdChunk, wmax - base);
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const uint32_t id = ids[beg + base + j];
            const float4* src = reinterpret_cast<const float4*>(pv + id);
            const float4 r0 = src[0], r1 = src[1], r2 = src[2];
            float4 a, b;
            make_rec(r0, r1, a, b);
            s_a[j] = a;
            s_b[j] = b;
            s_u[j] = make_float4(r0.z, r0.w, r1.x, 0.f);
            s_c[j] = r2.x;
            s_id[j] = id;
            s_rows[j] = reach_rows(a, b, qmax, tile_y0, TH);
        }
        __syncthreads();
        // this wave's list of the entries reaching its rows; partial sums of the
        // entries it does not visit stay zero
        uint16_t* const L = s_list[wid];
        const int nl = wave_list(s_rows, cnt, row_lo, row_hi, L);
        const int jlim = min(cnt, wave_walk - base);
        for (int j = threadIdx.x; j < cnt; j += NT)
#pragma unroll
            for (int c = 0; c < kG; ++c) s_part[c][j] = 0.f;
        __syncthreads();   // cleared before any wave adds into them
        // groups of four entries: per-lane gradients, then one reduce-scatter per component
        for (int i = 0; i < nl; i += 4) {
            const uint2 q = *reinterpret_cast<const uint2*>(L + i);
            const uint32_t qx = __builtin_amdgcn_readfirstlane(q.x), qy = __builtin_amdgcn_readfirstlane(q.y);
            const int js[4] = {(int)(qx & 0xffffu), (int)(qx >> 16), (int)(qy & 0xffffu), (int)(qy >> 16)};
            if (js[0] >= jlim) break;
            // per entry and lane, five values from which the nine gradient terms follow
            // at the reduction: w = T alpha, dL/dalpha G, dL/dq (0 where alpha is clamped), dx, dy
            float gw[4], go[4], gq[4], gx[4], gy[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) gw[u] = go[u] = gq[u] = gx[u] = gy[u] = 0.f;
            bool any = false;
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (i + u >= nl || js[u] >= jlim) break;
                const int j = js[u];
                if (base + j >= walk) continue;
                const float4 a = s_a[j];
                const float4 b = s_b[j];
                const Gauss e = eval_gauss(a, b, fx, fy);
                const float al = alpha_of(e, emin, amin, amax);
                if (al != 0.f) {
                    const float al0 = e.al0;
                    const float w = __fmul_rn(T, al);
                    const float cr = b.z, cg = b.w, cb = s_c[j];
                    Pr = add_weighted(Pr, w, cr);
                    Pg = add_weighted(Pg, w, cg);
                    Pb = add_weighted(Pb, w, cb);
                    const float inv = __builtin_amdgcn_rcpf(1.f - al);
                    const float dLda = gr * (T * cr - (PKr - Pr + Br) * inv) + gg * (T * cg - (PKg - Pg + Bg) * inv) +
                                       gb * (T * cb - (PKb - Pb + Bb) * inv);
                    gw[u] = w;
                    if (al0 < amax) {
                        go[u] = dLda * e.G;                      // dalpha/do = G
                        gq[u] = -0.5f * al0 * dLda;              // dL/dq
                        gx[u] = e.dx;
                        gy[u] = e.dy;
                    }
                    any = true;
                    T = next_T(T, al);
                }
            }
            if (__ballot(any) == 0) continue;
            const int jw = lane == 0 ? js[0] : lane == 1 ? js[1] : lane == 2 ? js[2] : js[3];
            const bool writer = lane < 4 && i + lane < nl && jw < jlim;
            // the mean2d terms 2 dL/dq (a dx + b dy), 2 dL/dq (b dx + c dy) are formed from
            // the sums of dL/dq dx and dL/dq dy with the entry's conic (a, b, c)
            float sq[9];
            {
                float t0[4], t1[4], t2[4], t3[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    t0[u] = gq[u] * gx[u];
                    t1[u] = gq[u] * gy[u];
                }
                sq[0] = wave_sum4(t0[0], t0[1], t0[2], t0[3]);
                sq[1] = wave_sum4(t1[0], t1[1], t1[2], t1[3]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    t2[u] = t0[u] * gx[u];
                    t3[u] = t0[u] * gy[u];
                    t0[u] = t1[u] * gy[u];
                }
                sq[2] = wave_sum4(t2[0], t2[1], t2[2], t2[3]);
                sq[3] = wave_sum4(t3[0], t3[1], t3[2], t3[3]);
                sq[4] = wave_sum4(t0[0], t0[1], t0[2], t0[3]);
                sq[5] = wave_sum4(go[0], go[1], go[2], go[3]);
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    t0[u] = gr * gw[u];
                    t1[u] = gg * gw[u];
                    t2[u] = gb * gw[u];
                }
                sq[6] = wave_sum4(t0[0], t0[1], t0[2], t0[3]);
                sq[7] = wave_sum4(t1[0], t1[1], t1[2], t1[3]);
                sq[8] = wave_sum4(t2[0], t2[1], t2[2], t2[3]);
            }
            if (writer) {
                const float4 cn = s_u[jw];   // conic a, b, c of the lane's entry
                const float gs[kG] = {2.f * (cn.x * sq[0] + cn.y * sq[1]), 2.f * (cn.y * sq[0] + cn.z * sq[1]),
                                      sq[2], 2.f * sq[3], sq[4], sq[5], sq[6], sq[7], sq[8]};
#pragma unroll
                for (int c = 0; c < kG; ++c)
                    if (gs[c] != 0.f) atomicAdd(&s_part[c][jw], gs[c]);
            }
        }
        __syncthreads();
        for (int e = threadIdx.x; e < cnt * kG; e += NT) {
            const int j = e / kG, c = e - j * kG;
            const float t = s_part[c][j];
            if (t != 0.f) unsafeAtomicAdd(grad2d + ((int64_t)v * N + s_id[j]) * kG + c, t);
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- projection backward (FP64)
// Term K of the Cartesian real SH basis (Y as in k_project) and its gradient
// with respect to the direction components, as compile-time expressions so
// that a fully unrolled loop over K keeps everything in registers.
template <int K>
__device__ inline void sh_term(double x, double y, double z, double& Y, double& Gx, double& Gy, double& Gz) {
    constexpr double c1 = 0.4886025119029199;
    constexpr double a2 = 1.0925484305920792, b2 = 0.31539156525252005, c2 = 0.5462742152960396;
    constexpr double a3 = 0.5900435899266435, b3 = 2.890611442640554, c3 = 0.4570457994644658,
                     d3 = 0.3731763325901154, e3 = 1.445305721320277;
    Gx = Gy = Gz = 0.0;
    if constexpr (K == 0) {
        Y = 0.28209479177387814;
    } else if constexpr (K == 1) {
        Y = -c1 * y; Gy = -c1;
    } else if constexpr (K == 2) {
        Y = c1 * z; Gz = c1;
    } else if constexpr (K == 3) {
        Y = -c1 * x; Gx = -c1;
    } else if constexpr (K == 4) {
        Y = a2 * x * y; Gx = a2 * y; Gy = a2 * x;
    } else if constexpr (K == 5) {
        Y = -a2 * y * z; Gy = -a2 * z; Gz = -a2 * y;
    } else if constexpr (K == 6) {
        Y = b2 * (2.0 * z * z - x * x - y * y); Gx = -2.0 * b2 * x; Gy = -2.0 * b2 * y; Gz = 4.0 * b2 * z;
    } else if constexpr (K == 7) {
        Y = -a2 * x * z; Gx = -a2 * z; Gz = -a2 * x;
    } else if constexpr (K == 8) {
        Y = c2 * (x * x - y * y); Gx = 2.0 * c2 * x; Gy = -2.0 * c2 * y;
    } else if constexpr (K == 9) {
        Y = -a3 * y * (3.0 * x * x - y * y); Gx = -6.0 * a3 * x * y; Gy = -3.0 * a3 * (x * x - y * y);
    } else if constexpr (K == 10) {
        Y = b3 * x * y * z; Gx = b3 * y * z; Gy = b3 * x * z; Gz = b3 * x * y;
    } else if constexpr (K == 11) {
        Y = -c3 * y * (4.0 * z * z - x * x - y * y);
        Gx = 2.0 * c3 * x * y; Gy = -c3 * (4.0 * z * z - x * x - 3.0 * y * y); Gz = -8.0 * c3 * y * z;
    } else if constexpr (K == 12) {
        Y = d3 * z * (2.0 * z * z - 3.0 * x * x - 3.0 * y * y);
        Gx = -6.0 * d3 * x * z; Gy = -6.0 * d3 * y * z; Gz = d3 * (6.0 * z * z - 3.0 * x * x - 3.0 * y * y);
    } else if constexpr (K == 13) {
        Y = -c3 * x * (4.0 * z * z - x * x - y * y);
        Gx = -c3 * (4.0 * z * z - 3.0 * x * x - y * y); Gy = 2.0 * c3 * x * y; Gz = -8.0 * c3 * x * z;
    } else if constexpr (K == 14) {
        Y = e3 * z * (x * x - y * y); Gx = 2.0 * e3 * x * z; Gy = -2.0 * e3 * y * z; Gz = e3 * (x * x - y * y);
    } else {
        Y = -a3 * x * (x * x - 3.0 * y * y); Gx = -3.0 * a3 * (x * x - y * y); Gy = 6.0 * a3 * x * y;
    }
}

// f(integral_constant<int, K>) for K = 0 .. N-1, unrolled at compile time
template <int K, int N, typename F>
__device__ inline void static_for(F&& f) {
    if constexpr (K < N) {
        f(std::integral_constant<int, K>{});
        static_for<K + 1, N>(f);
    }
}

// DEG: the SH degree in use (0..3), a template argument so that every SH loop is
// unrolled with compile-time indices (no register arrays indexed at run time).
template <int DEG>
__global__ __launch_bounds__(256) void k_project_bwd(int64_t N, int32_t v0, int32_t nv, CamBatch cams,
                                                     potr_config cfg, const float* __restrict__ means,
                                                     const float* __restrict__ scales,
                                                     const float* __restrict__ quats, const float* __restrict__ opac,
                                                     const float* __restrict__ sh, const float* __restrict__ grad2d,
                                                     float* __restrict__ d_means, float* __restrict__ d_scales,
                                                     float* __restrict__ d_quats, float* __restrict__ d_opac,
                                                     float* __restrict__ d_sh) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= N) return;
    const double mx = means[3 * i], my = means[3 * i + 1], mz = means[3 * i + 2];
    const double q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const double qn = sqrt(q0 * q0 + q1 * q1 + q2 * q2 + q3 * q3);
    if (!(qn > 0.0)) return;
    const double w = q0 / qn, x = q1 / qn, y = q2 / qn, z = q3 / qn;
    const double M0[9] = {1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y),
                          2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x),
                          2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)};
    const double s[3] = {scales[3 * i], scales[3 * i + 1], scales[3 * i + 2]};
    double Mm[9], Sg[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Mm[3 * r + k] = M0[3 * r + k] * s[k];
    for (int a = 0; a < 3; ++a)
        for (int b = a; b < 3; ++b) {
            const double v = Mm[3 * a] * Mm[3 * b] + Mm[3 * a + 1] * Mm[3 * b + 1] + Mm[3 * a + 2] * Mm[3 * b + 2];
            Sg[3 * a + b] = v;
            Sg[3 * b + a] = v;
        }
    constexpr int nsh = (DEG + 1) * (DEG + 1);
    const float* shp = sh + 48 * i;

    double gm[3] = {0, 0, 0}, gSig[9] = {0, 0, 0, 0, 0, 0, 0, 0, 0}, go = 0.0;
    float gsh[3 * nsh];
#pragma unroll
    for (int k = 0; k < 3 * nsh; ++k) gsh[k] = 0.f;
    bool touched = false;

    for (int vv = 0; vv < nv; ++vv) {
        const float* g2 = grad2d + ((int64_t)(v0 + vv) * N + i) * 9;
        const double gu = g2[0], gv = g2[1], gA = g2[2], gB = g2[3], gC = g2[4], gO = g2[5];
        const double gcol[3] = {g2[6], g2[7], g2[8]};
        if (gu == 0.0 && gv == 0.0 && gA == 0.0 && gB == 0.0 && gC == 0.0 && gO == 0.0 && gcol[0] == 0.0 &&
            gcol[1] == 0.0 && gcol[2] == 0.0)
            continue;
        touched = true;
        const potr_camera& c = cams.c[vv];
        double R[9];
        for (int k = 0; k < 9; ++k) R[k] = c.R[k];
        const double px = R[0] * mx + R[1] * my + R[2] * mz + (double)c.t[0];
        const double py = R[3] * mx + R[4] * my + R[5] * mz + (double)c.t[1];
        const double pz = R[6] * mx + R[7] * my + R[8] * mz + (double)c.t[2];
        const double fx = c.fx, fy = c.fy;
        const double limx = (double)cfg.jclamp * 0.5 * c.width / fx;
        const double limy = (double)cfg.jclamp * 0.5 * c.height / fy;
        const double rx = px / pz, ry = py / pz;
        const bool freex = rx > -limx && rx < limx, freey = ry > -limy && ry < limy;
        const double tx = fmin(limx, fmax(-limx, rx)), ty = fmin(limy, fmax(-limy, ry));
        const double j00 = fx / pz, j02 = -fx * tx / pz, j11 = fy / pz, j12 = -fy * ty / pz;
        const double T[6] = {j00 * R[0] + j02 * R[6], j00 * R[1] + j02 * R[7], j00 * R[2] + j02 * R[8],
                             j11 * R[3] + j12 * R[6], j11 * R[4] + j12 * R[7], j11 * R[5] + j12 * R[8]};
        double TS[6];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b)
                TS[3 * a + b] = T[3 * a] * Sg[b] + T[3 * a + 1] * Sg[3 + b] + T[3 * a + 2] * Sg[6 + b];
        const double cxx = TS[0] * T[0] + TS[1] * T[1] + TS[2] * T[2] + (double)cfg.eps2d;
        const double cxy = TS[0] * T[3] + TS[1] * T[4] + TS[2] * T[5];
        const double cyy = TS[3] * T[3] + TS[4] * T[4] + TS[5] * T[5] + (double)cfg.eps2d;
        const double det = cxx * cyy - cxy * cxy;
        const double Qa = cyy / det, Qb = -cxy / det, Qc = cxx / det;
        // conic -> cov2d: G_S = -Q G_Q Q, G_Q = [[gA, gB/2], [gB/2, gC]]
        const double h00 = gA * Qa + 0.5 * gB * Qb, h01 = gA * Qb + 0.5 * gB * Qc;
        const double h10 = 0.5 * gB * Qa + gC * Qb, h11 = 0.5 * gB * Qb + gC * Qc;
        const double S00 = -(Qa * h00 + Qb * h10), S01 = -(Qa * h01 + Qb * h11);
        const double S11 = -(Qb * h01 + Qc * h11);
        // cov2d = T Sigma T^T: G_Sigma = T^T G_S T, G_T = 2 G_S T Sigma
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b)
                gSig[3 * a + b] += T[a] * (S00 * T[b] + S01 * T[3 + b]) + T[3 + a] * (S01 * T[b] + S11 * T[3 + b]);
        double GT[6];
        for (int b = 0; b < 3; ++b) {
            GT[b] = 2.0 * (S00 * TS[b] + S01 * TS[3 + b]);
            GT[3 + b] = 2.0 * (S01 * TS[b] + S11 * TS[3 + b]);
        }
        // T = J R: G_J = G_T R^T (only the non-zero entries of J are needed)
        const double gj00 = GT[0] * R[0] + GT[1] * R[1] + GT[2] * R[2];
        const double gj02 = GT[0] * R[6] + GT[1] * R[7] + GT[2] * R[8];
        const double gj11 = GT[3] * R[3] + GT[4] * R[4] + GT[5] * R[5];
        const double gj12 = GT[3] * R[6] + GT[4] * R[7] + GT[5] * R[8];
        const double iz2 = 1.0 / (pz * pz);
        double gpx = 0.0, gpy = 0.0, gpz = 0.0;
        gpz += -gj00 * fx * iz2 - gj11 * fy * iz2;
        if (freex) gpx += -gj02 * fx * iz2;
        gpz += gj02 * fx * tx * iz2 * (freex ? 2.0 : 1.0);
        if (freey) gpy += -gj12 * fy * iz2;
        gpz += gj12 * fy * ty * iz2 * (freey ? 2.0 : 1.0);
        // pixel centre u = fx x/z + cx, v = fy y/z + cy
        gpx += gu * fx / pz;
        gpy += gv * fy / pz;
        gpz += -(gu * fx * px + gv * fy * py) * iz2;
        gm[0] += R[0] * gpx + R[3] * gpy + R[6] * gpz;
        gm[1] += R[1] * gpx + R[4] * gpy + R[7] * gpz;
        gm[2] += R[2] * gpx + R[5] * gpy + R[8] * gpz;
        go += gO;
        // colour along d = (mu - eye) / |mu - eye|, clamped at 0
        const double ex = -(R[0] * c.t[0] + R[3] * c.t[1] + R[6] * c.t[2]);
        const double ey = -(R[1] * c.t[0] + R[4] * c.t[1] + R[7] * c.t[2]);
        const double ez = -(R[2] * c.t[0] + R[5] * c.t[1] + R[8] * c.t[2]);
        double ux = mx - ex, uy = my - ey, uz = mz - ez;
        const double un = sqrt(ux * ux + uy * uy + uz * uz);
        const double dx = ux / un, dy = uy / un, dz = uz / un;
        // colour before the clamp, per channel; the clamp passes the gradient
        // where it is positive
        double pre[3] = {0.5, 0.5, 0.5};
        static_for<0, nsh>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            double Yk, gxk, gyk, gzk;
            sh_term<k>(dx, dy, dz, Yk, gxk, gyk, gzk);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) pre[ch] += (double)shp[3 * k + ch] * Yk;
        });
        double gc[3];
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) gc[ch] = (pre[ch] > 0.0) ? gcol[ch] : 0.0;
        double gdx = 0.0, gdy = 0.0, gdz = 0.0;
        static_for<0, nsh>([&](auto kc) {
            constexpr int k = decltype(kc)::value;
            double Yk, Gxk, Gyk, Gzk;
            sh_term<k>(dx, dy, dz, Yk, Gxk, Gyk, Gzk);
#pragma unroll
            for (int ch = 0; ch < 3; ++ch) {
                gsh[3 * k + ch] += (float)(gc[ch] * Yk);
                const double gy = gc[ch] * (double)shp[3 * k + ch];
                gdx += gy * Gxk;
                gdy += gy * Gyk;
                gdz += gy * Gzk;
            }
        });
        const double dot = gdx * dx + gdy * dy + gdz * dz;
        gm[0] += (gdx - dx * dot) / un;
        gm[1] += (gdy - dy * dot) / un;
        gm[2] += (gdz - dz * dot) / un;
    }
    if (!touched) return;
    // Sigma = M M^T with M = R(q) diag(s)
    double GM[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b)
            GM[3 * a + b] = (gSig[3 * a] + gSig[a]) * Mm[b] + (gSig[3 * a + 1] + gSig[3 + a]) * Mm[3 + b] +
                            (gSig[3 * a + 2] + gSig[6 + a]) * Mm[6 + b];
    double GR[9];
    double gs[3] = {0, 0, 0};
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            gs[k] += GM[3 * r + k] * M0[3 * r + k];
            GR[3 * r + k] = GM[3 * r + k] * s[k];
        }
    const double gw = 2 * (-z * GR[1] + y * GR[2] + z * GR[3] - x * GR[5] - y * GR[6] + x * GR[7]);
    const double gx = 2 * (y * GR[1] + z * GR[2] + y * GR[3] - 2 * x * GR[4] - w * GR[5] + z * GR[6] + w * GR[7] -
                           2 * x * GR[8]);
    const double gy = 2 * (-2 * y * GR[0] + x * GR[1] + w * GR[2] + x * GR[3] + z * GR[5] - w * GR[6] + z * GR[7] -
                           2 * y * GR[8]);
    const double gz = 2 * (-2 * z * GR[0] - w * GR[1] + x * GR[2] + w * GR[3] - 2 * z * GR[4] + y * GR[5] +
                           x * GR[6] + y * GR[7]);
    const double dq = gw * w + gx * x + gy * y + gz * z;
    d_means[3 * i] += (float)gm[0];
    d_means[3 * i + 1] += (float)gm[1];
    d_means[3 * i + 2] += (float)gm[2];
    for (int k = 0; k < 3; ++k) d_scales[3 * i + k] += (float)gs[k];
    d_quats[4 * i] += (float)((gw - w * dq) / qn);
    d_quats[4 * i + 1] += (float)((gx - x * dq) / qn);
    d_quats[4 * i + 2] += (float)((gy - y * dq) / qn);
    d_quats[4 * i + 3] += (float)((gz - z * dq) / qn);
    d_opac[i] += (float)go;
#pragma unroll
    for (int k = 0; k < nsh * 3; ++k) d_sh[48 * i + k] += gsh[k];
}

__global__ void k_fill_f32(float* p, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.f;
}

template <int TW, int TH>
potr_status blend_bwd_shape(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg,
                            const potr_proj* proj, const uint32_t* ids, const int32_t* ranges, const float* p_final,
                            const float* t_final, const int32_t* n_walk, const float* dL, float* grad2d,
                            hipStream_t s) {
    const int txs = tiles_x(c, cfg), tpv = txs * tiles_y(c, cfg);
    hipLaunchKernelGGL((k_blend_bwd<TW, TH>), dim3(tpv, V), dim3(TW * TH), 0, s, N, c.width, c.height, txs, tpv, cfg,
                       proj, ids, ranges, p_final, t_final, n_walk, dL, grad2d);
    return check_launch("k_blend_bwd");
}

}  // namespace

potr_status launch_blend_backward(int64_t N, int32_t V, const potr_camera& c, const potr_config& cfg,
                                  const potr_proj* proj, const uint32_t* ids, const int32_t* ranges,
                                  const float* p_final, const float* t_final, const int32_t* n_walk, const float* dL,
                                  float* grad2d, hipStream_t s) {
    if (cfg.tile_w == 16 && cfg.tile_h == 16)
        return blend_bwd_shape<16, 16>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, dL, grad2d, s);
    if (cfg.tile_w == 8 && cfg.tile_h == 8)
        return blend_bwd_shape<8, 8>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, dL, grad2d, s);
    if (cfg.tile_w == 32 && cfg.tile_h == 8)
        return blend_bwd_shape<32, 8>(N, V, c, cfg, proj, ids, ranges, p_final, t_final, n_walk, dL, grad2d, s);
    return fail(POTR_EUNSUPPORTED, "tile %dx%d not built", cfg.tile_w, cfg.tile_h);
}

potr_status launch_project_backward(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                                    const float* means, const float* scales, const float* quats, const float* opac,
                                    const float* sh, const float* grad2d, float* d_means, float* d_scales,
                                    float* d_quats, float* d_opac, float* d_sh, hipStream_t s) {
    if (N == 0) return POTR_OK;
    const dim3 grid((unsigned)ceil_div(N, 256));
    for (int32_t v0 = 0; v0 < V; v0 += kViewsPerLaunch) {
        const int32_t nv = V - v0 < kViewsPerLaunch ? V - v0 : kViewsPerLaunch;
        CamBatch cb;
        for (int k = 0; k < nv; ++k) cb.c[k] = cams[v0 + k];
        for (int k = nv; k < kViewsPerLaunch; ++k) cb.c[k] = cams[v0];
        switch (cfg.sh_degree) {
            case 0:
                hipLaunchKernelGGL(k_project_bwd<0>, grid, dim3(256), 0, s, N, v0, nv, cb, cfg, means, scales, quats,
                                   opac, sh, grad2d, d_means, d_scales, d_quats, d_opac, d_sh);
                break;
            case 1:
                hipLaunchKernelGGL(k_project_bwd<1>, grid, dim3(256), 0, s, N, v0, nv, cb, cfg, means, scales, quats,
                                   opac, sh, grad2d, d_means, d_scales, d_quats, d_opac, d_sh);
                break;
            case 2:
                hipLaunchKernelGGL(k_project_bwd<2>, grid, dim3(256), 0, s, N, v0, nv, cb, cfg, means, scales, quats,
                                   opac, sh, grad2d, d_means, d_scales, d_quats, d_opac, d_sh);
                break;
            default:
                hipLaunchKernelGGL(k_project_bwd<3>, grid, dim3(256), 0, s, N, v0, nv, cb, cfg, means, scales, quats,
                                   opac, sh, grad2d, d_means, d_scales, d_quats, d_opac, d_sh);
                break;
        }
        potr_status st = check_launch("k_project_bwd");
        if (st != POTR_OK) return st;
    }
    return POTR_OK;
}

potr_status launch_zero(float* p, int64_t n, hipStream_t s) {
    if (n <= 0) return POTR_OK;
    hipLaunchKernelGGL(k_fill_f32, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, p, n);
    return check_launch("k_fill_f32");
}

}  // namespace potr
