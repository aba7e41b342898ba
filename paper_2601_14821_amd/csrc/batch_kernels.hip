// Small kernels of the batch runtime: pair counting for planning, the L1 loss
// gradient of the fine-tuning step and the capacity check after a run.
#include "common.h"

namespace potr {
namespace {

__global__ void k_zero_counts(int64_t* c, int32_t n) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) c[i] = 0;
}

// counts[v] += sum of tiles_touched over the N splats of view v: one device
// atomic per block (atomics on one word serialise, so there are few blocks)
__global__ __launch_bounds__(256) void k_sum_tiles(const int32_t* __restrict__ tt, int64_t N,
                                                   int64_t* __restrict__ counts) {
    __shared__ int64_t s_w[4];
    const int v = blockIdx.y;
    int64_t acc = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < N; i += (int64_t)gridDim.x * blockDim.x)
        acc += tt[(int64_t)v * N + i];
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if ((threadIdx.x & 63) == 0) s_w[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
        const int64_t b = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        if (b != 0) atomicAdd((unsigned long long*)&counts[v], (unsigned long long)b);
    }
}

__global__ void k_check_overflow(const int64_t* __restrict__ n_pairs, const int64_t* __restrict__ caps, int32_t n,
                                 int32_t* __restrict__ flag) {
    if (threadIdx.x != 0) return;
    int32_t bad = 0;
    for (int32_t j = 0; j < n; ++j) bad += (n_pairs[j] > caps[j] || n_pairs[j] < 0) ? 1 : 0;
    *flag = bad;
}

// dL/dimage of L = w * sum |image - target|: w * sign(image - target), sign(0) = 0.
__global__ __launch_bounds__(256) void k_l1_grad(const float* __restrict__ image, const float* __restrict__ target,
                                                 int64_t n, float w, float* __restrict__ dl) {
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const float d = image[i] - target[i];
        dl[i] = d > 0.f ? w : (d < 0.f ? -w : 0.f);
    }
}

}  // namespace

potr_status launch_l1_grad(const float* image, const float* target, int64_t n, float w, float* dl, hipStream_t s) {
    if (n <= 0) return POTR_OK;
    const int64_t b = ceil_div(n, 256);
    hipLaunchKernelGGL(k_l1_grad, dim3((unsigned)(b < 8192 ? b : 8192)), dim3(256), 0, s, image, target, n, w, dl);
    return check_launch("k_l1_grad");
}

potr_status launch_count_pairs(int64_t N, int32_t V, const potr_camera* cams, const potr_config& cfg,
                               const float* means, const float* scales, const float* quats, const float* opac,
                               const float* sh, potr_proj* proj, int32_t* tt, int64_t* counts, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_counts, dim3(1), dim3(256), 0, s, counts, V);
    potr_status st = check_launch("k_zero_counts");
    if (st != POTR_OK) return st;
    st = launch_project(N, V, cams, cfg, means, scales, quats, opac, sh, proj, tt, s);
    if (st != POTR_OK || N == 0) return st;
    int64_t blocks = ceil_div(N, 256 * 16);   // at least 16 values per thread, at most 128 atomics per view
    if (blocks > 128) blocks = 128;
    hipLaunchKernelGGL(k_sum_tiles, dim3((unsigned)blocks, V), dim3(256), 0, s, tt, N, counts);
    return check_launch("k_sum_tiles");
}

potr_status launch_check_overflow(const int64_t* n_pairs, const int64_t* caps, int32_t n, int32_t* flag,
                                  hipStream_t s) {
    hipLaunchKernelGGL(k_check_overflow, dim3(1), dim3(64), 0, s, n_pairs, caps, n, flag);
    return check_launch("k_check_overflow");
}

}  // namespace potr
