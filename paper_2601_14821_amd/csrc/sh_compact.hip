// Spherical-harmonics energy compaction (paper Sec. 4.4): per splat, new
// lighting coefficients from an importance-weighted ridge regression of the
// colours the training cameras see, in YCoCg, with parallel columns dropped
// and a second pass without the coefficients the first one left almost zero.
//
// Per splat the regression only needs the weighted Gram matrix
// G = Y_w^T Y_w (Y_w: the SH basis at the camera directions, rows scaled by the
// camera weights), because the colours are C = Y L, so the right-hand side is
// Y_w^T C_w = G L and the cosines between columns are G_ij / sqrt(G_ii G_jj).
//   k_sh_eyes   camera centres -R^T t (FP64) into the workspace;
//   k_sh_seen   one thread per splat, coalesced over the importance rows: its
//               largest camera importance; a splat no camera sees gets its
//               output (the DC, AC 0) here, the others go to a list (one
//               atomic per wave), so the two kernels below run full waves of
//               seen splats however sparse they are;
//   k_sh_gram   one wave per listed splat: G by FP64 matrix-core products,
//               4 cameras per v_mfma_f64_16x16x4 (the wave evaluates the basis
//               of 64 cameras at once, one per lane, stages the weighted values
//               in LDS and feeds them to the matrix core in its operand layout),
//               upper triangle to the workspace;
//   k_sh_solve  one thread per listed splat: column selection, the right-hand
//               sides of the three channels in one pass over G, then per channel
//               the two ridge solves by Cholesky in the thread's LDS (Co and Cg
//               have the same weight, so their first solves share a factor),
//               back to RGB.
// A splat's result depends only on its own data, so the list's order (set by
// the atomics) does not change any output. All arithmetic is FP64.
#include "common.h"
#include "sh_basis.h"
#include "sh_compact.h"

namespace potr {
namespace {

typedef double f64x4 __attribute__((ext_vector_type(4)));

constexpr int kPacked = 136;                 // upper triangle of 16 x 16
constexpr int kSplatStride = kPacked + 1;    // per splat: G, then its largest camera importance
constexpr int kSolveThreads = 64;
constexpr int kFStride = 137;                // doubles per thread of the factor in LDS (odd: spreads banks)
constexpr int64_t kListBlocks = 8192;        // grid of the list kernels (they stride over the seen count)

__device__ inline int packed_upper(int i, int j) {   // i <= j
    return i * 16 - (i * (i - 1)) / 2 + (j - i);
}

__global__ void k_sh_eyes(CamBatch cams, int32_t v0, int32_t nv, double* __restrict__ eyes) {
    const int k = threadIdx.x;
    if (k >= nv) return;
    const potr_camera& c = cams.c[k];
    double e[3];
    for (int a = 0; a < 3; ++a)
        e[a] = -((double)c.R[a] * (double)c.t[0] + (double)c.R[3 + a] * (double)c.t[1] +
                 (double)c.R[6 + a] * (double)c.t[2]);
    for (int a = 0; a < 3; ++a) eyes[3 * (int64_t)(v0 + k) + a] = e[a];
}

__global__ void k_sh_clear(uint32_t* n_seen) { *n_seen = 0u; }

__global__ __launch_bounds__(256) void k_sh_seen(int64_t N, int32_t V, const float* __restrict__ sh,
                                                 const float* __restrict__ imp, int64_t stride,
                                                 double* __restrict__ gws, uint32_t* __restrict__ n_seen,
                                                 int32_t* __restrict__ list, float* __restrict__ sh_out) {
    __shared__ uint8_t s_seen[256];
    const int64_t k0 = (int64_t)blockIdx.x * 256;
    const int64_t k = k0 + threadIdx.x;
    float m = 0.f;
    if (k < N) {   // four running maxima keep four loads in flight
        float m1 = 0.f, m2 = 0.f, m3 = 0.f;
        const float* col = imp + k;
        int32_t v = 0;
        for (; v + 4 <= V; v += 4) {
            m = fmaxf(m, col[(int64_t)v * stride]);
            m1 = fmaxf(m1, col[(int64_t)(v + 1) * stride]);
            m2 = fmaxf(m2, col[(int64_t)(v + 2) * stride]);
            m3 = fmaxf(m3, col[(int64_t)(v + 3) * stride]);
        }
        for (; v < V; ++v) m = fmaxf(m, col[(int64_t)v * stride]);
        m = fmaxf(fmaxf(m, m1), fmaxf(m2, m3));
    }
    const bool seen = k < N && m > 0.f;
    const uint64_t bal = __ballot(seen);
    if (bal != 0) {
        const int lane = threadIdx.x & 63;
        const int lead = __ffsll((long long)bal) - 1;
        uint32_t base = 0;
        if (lane == lead) base = atomicAdd(n_seen, (uint32_t)__popcll(bal));
        base = __shfl(base, lead, 64);
        if (seen) list[base + __popcll(bal & ((uint64_t(1) << lane) - 1))] = (int32_t)k;
    }
    if (seen) gws[k * kSplatStride + kPacked] = (double)m;
    s_seen[threadIdx.x] = seen ? 1 : 0;
    __syncthreads();
    // a splat no camera sees keeps its DC, the rest 0: the block writes the
    // outputs of its unseen splats together, consecutive threads on
    // consecutive floats
    const int64_t nk = N - k0 < 256 ? N - k0 : 256;
    for (int e = threadIdx.x; e < nk * 48; e += 256) {
        const int j = e / 48, c = e - 48 * j;
        if (s_seen[j]) continue;
        sh_out[48 * k0 + e] = c < 3 ? sh[48 * k0 + e] : 0.f;
    }
}

// One wave (64 threads) per listed splat.
__global__ __launch_bounds__(64) void k_sh_gram(int32_t V, int degree, const double* __restrict__ eyes,
                                                const float* __restrict__ means, const float* __restrict__ imp,
                                                int64_t stride, double* __restrict__ gws,
                                                const uint32_t* __restrict__ n_seen,
                                                const int32_t* __restrict__ list) {
    __shared__ double sy[64 * 17];   // weighted basis of 64 cameras (17: padding)
    const uint32_t n = *n_seen;
    const int lane = threadIdx.x;
    for (uint32_t it = blockIdx.x; it < n; it += gridDim.x) {
        const int64_t k = list[it];
        double* G = gws + k * kSplatStride;
        const double imax = G[kPacked];   // the splat's largest camera importance (> 0)
        const double mx = means[3 * k], my = means[3 * k + 1], mz = means[3 * k + 2];
        f64x4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int v0 = 0; v0 < V; v0 += 64) {
            const int v = v0 + lane;
            double y[16];
#pragma unroll
            for (int i = 0; i < 16; ++i) y[i] = 0.0;
            double w = 0.0;
            if (v < V) {
                w = (double)imp[(int64_t)v * stride + k] / imax;
                double dx = mx - eyes[3 * v], dy = my - eyes[3 * v + 1], dz = mz - eyes[3 * v + 2];
                const double r = __builtin_sqrt(dx * dx + dy * dy + dz * dz);
                dx /= r;
                dy /= r;
                dz /= r;
                sh_basis_d3(dx, dy, dz, degree, y);
            }
#pragma unroll
            for (int i = 0; i < 16; ++i) sy[lane * 17 + i] = w * y[i];
            __syncthreads();
            // 16 products of 4 cameras each: lane l supplies basis l % 16 of camera l / 16
            // as both A[i][c] and B[c][j] (Y_w^T is A, Y_w is B)
            const int cams = min(64, V - v0);
            for (int c0 = 0; c0 < cams; c0 += 4) {
                const double a = sy[(c0 + lane / 16) * 17 + (lane % 16)];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, a, acc, 0, 0, 0);
            }
            __syncthreads();
        }
        // the product's layout (measured): D[i][j] is register i / 4 of lane j + 16 (i % 4)
        const int j = lane % 16;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int i = lane / 16 + 4 * r;
            if (i <= j) G[packed_upper(i, j)] = acc[r];
        }
    }
}

struct Solver {
    const double* G;   // this splat's packed upper triangle
    double* F;         // this thread's factor (packed lower, row-major)
    int M;

    __device__ double g(int i, int j) const { return i <= j ? G[packed_upper(i, j)] : G[packed_upper(j, i)]; }

    // Cholesky of G + lam diag(0, 1, .., 1) over the columns in `mask` (the
    // others become identity rows, so their unknowns solve to 0).
    __device__ void factor(uint32_t mask, double lam) {
        for (int i = 0; i < M; ++i) {
            const int ri = (i * (i + 1)) / 2;
            const bool ki = (mask >> i) & 1u;
            for (int j = 0; j <= i; ++j) {
                const bool kj = (mask >> j) & 1u;
                if (!ki || !kj) {
                    F[ri + j] = (i == j) ? 1.0 : 0.0;
                    continue;
                }
                double s = g(i, j) + ((i == j && i > 0) ? lam : 0.0);
                const int rj = (j * (j + 1)) / 2;
                for (int q = 0; q < j; ++q) s -= F[ri + q] * F[rj + q];
                F[ri + j] = (i == j) ? __builtin_sqrt(s) : s / F[rj + j];
            }
        }
    }

    // x = (L L^T)^-1 b over the mask (rows outside it give 0); b and x stay in
    // registers (every index below is a compile-time constant).
    __device__ __forceinline__ void solve(uint32_t mask, const double (&b)[16], double (&x)[16]) const {
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            if (i >= M) break;
            const int ri = (i * (i + 1)) / 2;
            double s = ((mask >> i) & 1u) ? b[i] : 0.0;
#pragma unroll
            for (int q = 0; q < i; ++q) s -= F[ri + q] * x[q];
            x[i] = s / F[ri + i];
        }
#pragma unroll
        for (int i = 15; i >= 0; --i) {
            if (i >= M) continue;
            double s = x[i];
#pragma unroll
            for (int q = i + 1; q < 16; ++q)
                if (q < M) s -= F[(q * (q + 1)) / 2 + i] * x[q];
            x[i] = s / F[(i * (i + 1)) / 2 + i];
        }
    }
};

// The second ridge pass: AC coefficients below tau are forced to 0 and the
// rest solved again (nothing to do when none is dropped). The factor holds
// (kept, lam) on entry; it is replaced only when the pass runs.
__device__ __forceinline__ void second_pass(Solver& S, uint32_t kept, double lam, double tau, const double (&b)[16],
                            double (&x)[16]) {
    uint32_t kept2 = kept;
#pragma unroll
    for (int i = 1; i < 16; ++i)
        if (i < S.M && ((kept >> i) & 1u) && fabs(x[i]) < tau) kept2 &= ~(1u << i);
    if (kept2 == kept) return;
    S.factor(kept2, lam);
    S.solve(kept2, b, x);
}

__global__ __launch_bounds__(kSolveThreads) void k_sh_solve(int degree, const float* __restrict__ sh,
                                                            double* __restrict__ gws, ShCompactParams p,
                                                            const uint32_t* __restrict__ n_seen,
                                                            const int32_t* __restrict__ list,
                                                            float* __restrict__ sh_out) {
    __shared__ double sF[kSolveThreads * kFStride];
    const uint32_t n = *n_seen;
    const int M = (degree + 1) * (degree + 1);
    for (uint32_t it = blockIdx.x * kSolveThreads + threadIdx.x; it < n; it += gridDim.x * kSolveThreads) {
        const int64_t k = list[it];
        const double* G = gws + k * kSplatStride;
        const float* L = sh + 48 * k;
        float* out = sh_out + 48 * k;
        Solver S{G, sF + threadIdx.x * kFStride, M};
        // columns: the DC, then each AC column not parallel to a kept one before it
        uint32_t kept = 1u;
        for (int i = 1; i < M; ++i) {
            const double gii = S.g(i, i);
            if (!(gii > 0.0)) continue;
            bool par = false;
            for (int j = 0; j < i; ++j) {
                if (!((kept >> j) & 1u)) continue;
                const double c = fabs(S.g(i, j)) / (__builtin_sqrt(gii) * __builtin_sqrt(S.g(j, j)));
                par = par || c > p.alpha;
            }
            if (!par) kept |= 1u << i;
        }
        // the coefficients in YCoCg and the right-hand sides G L of the three
        // channels, in one pass over the packed upper triangle
        double l0[16], l1[16], l2[16], b0[16], b1[16], b2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double R = L[3 * i], Gc = L[3 * i + 1], B = L[3 * i + 2];
            l0[i] = 0.25 * R + 0.5 * Gc + 0.25 * B;
            l1[i] = 0.5 * R - 0.5 * B;
            l2[i] = -0.25 * R + 0.5 * Gc - 0.25 * B;
            b0[i] = b1[i] = b2[i] = 0.0;
        }
#pragma unroll
        for (int i = 0; i < 16; ++i)
#pragma unroll
            for (int j = 0; j < 16; ++j) {
                if (j < i || j >= M) continue;
                const double g = G[packed_upper(i, j)];
                b0[i] += g * l0[j];
                b1[i] += g * l1[j];
                b2[i] += g * l2[j];
                if (j != i) {
                    b0[j] += g * l0[i];
                    b1[j] += g * l1[i];
                    b2[j] += g * l2[i];
                }
            }
        // Y with lam; Co and Cg share 3 lam, so their first solves share one
        // factorization (both are taken before either second pass refactors)
        double x0[16], x1[16], x2[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) x0[i] = x1[i] = x2[i] = 0.0;
        S.factor(kept, p.lam);
        S.solve(kept, b0, x0);
        second_pass(S, kept, p.lam, p.tau, b0, x0);
        S.factor(kept, 3.0 * p.lam);
        S.solve(kept, b1, x1);
        S.solve(kept, b2, x2);
        second_pass(S, kept, 3.0 * p.lam, p.tau, b1, x1);
        second_pass(S, kept, 3.0 * p.lam, p.tau, b2, x2);
#pragma unroll
        for (int i = 0; i < 16; ++i) {
            const double Yv = i < M ? x0[i] : 0.0, Co = i < M ? x1[i] : 0.0, Cg = i < M ? x2[i] : 0.0;
            out[3 * i] = (float)(Yv + Co - Cg);
            out[3 * i + 1] = (float)(Yv + Cg);
            out[3 * i + 2] = (float)(Yv - Co - Cg);
        }
    }
}

}  // namespace

// Workspace: camera centres [V,3] | seen count | seen list [N] | per splat
// kSplatStride doubles (G, then the largest importance).
size_t sh_compact_workspace_bytes(int64_t N, int32_t V) {
    return align_up((size_t)V * 3 * 8) + align_up(sizeof(uint32_t)) + align_up((size_t)N * 4) +
           (size_t)N * kSplatStride * 8;
}

potr_status launch_sh_compact(int64_t N, int32_t V, const potr_camera* cams, int degree, const float* means,
                              const float* sh, const float* imp, int64_t stride, const ShCompactParams& p,
                              void* ws, float* sh_out, hipStream_t s) {
    char* w = (char*)ws;
    double* eyes = (double*)w;
    w += align_up((size_t)V * 3 * 8);
    uint32_t* n_seen = (uint32_t*)w;
    w += align_up(sizeof(uint32_t));
    int32_t* list = (int32_t*)w;
    w += align_up((size_t)N * 4);
    double* gws = (double*)w;
    for (int32_t v0 = 0; v0 < V; v0 += kViewsPerLaunch) {
        const int32_t nv = V - v0 < kViewsPerLaunch ? V - v0 : kViewsPerLaunch;
        CamBatch cb{};
        for (int32_t k = 0; k < nv; ++k) cb.c[k] = cams[v0 + k];
        hipLaunchKernelGGL(k_sh_eyes, dim3(1), dim3(kViewsPerLaunch), 0, s, cb, v0, nv, eyes);
    }
    potr_status st = check_launch("k_sh_eyes");
    if (st != POTR_OK || N == 0) return st;
    // the seen count stays on the device: the two list kernels stride over it
    hipLaunchKernelGGL(k_sh_clear, dim3(1), dim3(1), 0, s, n_seen);
    hipLaunchKernelGGL(k_sh_seen, dim3((unsigned)((N + 255) / 256)), dim3(256), 0, s, N, V, sh, imp, stride, gws,
                       n_seen, list, sh_out);
    st = check_launch("k_sh_seen");
    if (st != POTR_OK) return st;
    const int64_t gram_blocks = N < kListBlocks ? N : kListBlocks;
    hipLaunchKernelGGL(k_sh_gram, dim3((unsigned)gram_blocks), dim3(64), 0, s, V, degree, eyes, means, imp, stride,
                       gws, n_seen, list);
    st = check_launch("k_sh_gram");
    if (st != POTR_OK) return st;
    const int64_t sb = (N + kSolveThreads - 1) / kSolveThreads;
    hipLaunchKernelGGL(k_sh_solve, dim3((unsigned)(sb < kListBlocks ? sb : kListBlocks)), dim3(kSolveThreads), 0, s,
                       degree, sh, gws, p, n_seen, list, sh_out);
    return check_launch("k_sh_solve");
}

}  // namespace potr
