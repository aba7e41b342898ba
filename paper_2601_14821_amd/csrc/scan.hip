// Device-wide exclusive scans (reduce -> scan of block sums -> downsweep).
#include "common.h"

namespace potr {
namespace {

template <typename T>
__device__ inline T wave_inclusive_scan(T x) {
    const int lane = threadIdx.x & 63;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        T y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

// Exclusive block scan of one value per thread (blockDim = kScanThreads).
template <typename T>
__device__ inline T block_exclusive_scan(T x, T* total) {
    __shared__ T warp_sums[kScanThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(x);
    if (lane == 63) warp_sums[w] = inc;
    __syncthreads();
    T base = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kScanThreads / 64; ++k) {
        T v = warp_sums[k];
        if (k < w) base += v;
        all += v;
    }
    __syncthreads();
    if (total) *total = all;
    return base + inc - x;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_reduce(const TI* __restrict__ in, int64_t n,
                                                              TO* __restrict__ block_sums) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    TO acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t e = base + (int64_t)k * kScanThreads + threadIdx.x;
        if (e < n) acc += (TO)in[e];
    }
    TO tot;
    block_exclusive_scan<TO>(acc, &tot);
    if (threadIdx.x == 0) block_sums[blockIdx.x] = tot;
}

// Single block: exclusive scan of nb block sums in place; writes the grand total.
template <typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_top(TO* sums, int64_t nb, TO* total) {
    TO carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t e = base + threadIdx.x;
        TO x = e < nb ? sums[e] : (TO)0;
        TO tot;
        TO ex = block_exclusive_scan<TO>(x, &tot);
        if (e < nb) sums[e] = carry + ex;
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kScanThreads) void k_scan_down(const TI* in, int64_t n, const TO* __restrict__ block_sums,
                                                            TO* out) {
    const int64_t base = (int64_t)blockIdx.x * kScanTile;
    // blocked arrangement: thread t owns items [t*kScanItems, (t+1)*kScanItems)
    TO v[kScanItems];
    TO acc = 0;
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t e = base + (int64_t)threadIdx.x * kScanItems + k;
        v[k] = e < n ? (TO)in[e] : (TO)0;
        acc += v[k];
    }
    TO tot;
    TO run = block_exclusive_scan<TO>(acc, &tot) + block_sums[blockIdx.x];
#pragma unroll
    for (int k = 0; k < kScanItems; ++k) {
        const int64_t e = base + (int64_t)threadIdx.x * kScanItems + k;
        const TO x = v[k];
        if (e < n) out[e] = run;
        run += x;
    }
}

// Whole scan in one workgroup of 1024 threads for inputs of at most one tile
// (1024 x 8 items): one launch instead of three.
constexpr int kOneThreads = 1024, kOneItems = 8;

template <typename T>
__device__ inline T block_exclusive_scan_1024(T x, T* total) {
    __shared__ T warp_sums[kOneThreads / 64];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T inc = wave_inclusive_scan(x);
    if (lane == 63) warp_sums[w] = inc;
    __syncthreads();
    T base = 0, all = 0;
#pragma unroll
    for (int k = 0; k < kOneThreads / 64; ++k) {
        T v = warp_sums[k];
        if (k < w) base += v;
        all += v;
    }
    __syncthreads();
    *total = all;
    return base + inc - x;
}

template <typename TI, typename TO>
__global__ __launch_bounds__(kOneThreads) void k_scan_one(const TI* in, int64_t n, TO* out, TO* total) {
    TO carry = 0;
    for (int64_t base = 0; base < n; base += (int64_t)kOneThreads * kOneItems) {
        TO v[kOneItems];
        TO acc = 0;
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            const int64_t e = base + (int64_t)threadIdx.x * kOneItems + k;
            v[k] = e < n ? (TO)in[e] : (TO)0;
            acc += v[k];
        }
        TO tot;
        TO run = carry + block_exclusive_scan_1024<TO>(acc, &tot);
#pragma unroll
        for (int k = 0; k < kOneItems; ++k) {
            const int64_t e = base + (int64_t)threadIdx.x * kOneItems + k;
            const TO x = v[k];
            if (e < n) out[e] = run;
            run += x;
        }
        carry += tot;
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <typename TI, typename TO>
potr_status scan_impl(const TI* in, TO* out, int64_t n, TO* total, void* tmp, hipStream_t s) {
    TO* sums = reinterpret_cast<TO*>(tmp);
    if (n > 0 && n <= (int64_t)kOneThreads * kOneItems) {
        hipLaunchKernelGGL((k_scan_one<TI, TO>), dim3(1), dim3(kOneThreads), 0, s, in, n, out, total);
        return check_launch("k_scan_one");
    }
    if (n <= 0) {
        if (total) {
            hipLaunchKernelGGL(k_scan_top<TO>, dim3(1), dim3(kScanThreads), 0, s, sums, (int64_t)0, total);
            return check_launch("k_scan_top");
        }
        return POTR_OK;
    }
    const int64_t nb = ceil_div(n, kScanTile);
    hipLaunchKernelGGL((k_scan_reduce<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n, sums);
    hipLaunchKernelGGL(k_scan_top<TO>, dim3(1), dim3(kScanThreads), 0, s, sums, nb, total);
    hipLaunchKernelGGL((k_scan_down<TI, TO>), dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, n,
                       (const TO*)sums, out);
    return check_launch("scan");
}

}  // namespace

size_t scan_tmp_bytes(int64_t n) { return align_up((size_t)(ceil_div(n > 0 ? n : 1, kScanTile) + 1) * 8); }

potr_status scan_i32_to_i64(const int32_t* in, int64_t* out, int64_t n, int64_t* total, void* tmp,
                            hipStream_t s) {
    return scan_impl<int32_t, int64_t>(in, out, n, total, tmp, s);
}

potr_status scan_u32(const uint32_t* in, uint32_t* out, int64_t n, void* tmp, hipStream_t s) {
    return scan_impl<uint32_t, uint32_t>(in, out, n, nullptr, tmp, s);
}

}  // namespace potr
