// One iteration of the pruning controller (paper Sec. 4.3) on the device, and
// the compaction of the survivors.
//
// The choice: candidates are the splats with dMSE_k < dMSE_MAX; the budget is
// the candidates' importance over the iterations still to run; candidates are
// taken in ascending order of m(dMSE_k / dMSE_MAX) (ties by index) until the
// importance taken reaches the budget. Instead of sorting, the cut is found by a
// radix select over the 96-bit composite (FP64 bits of m, splat index): per 8-bit
// digit one histogram pass sums, per digit value, the importance (as exact
// integers) of the candidates still in the current region, and one single-block
// pass picks the digit where the running sum reaches the budget. After 12
// digits the region is one splat, the last one removed; everything before it in
// the order is removed with it. Every pass recomputes the keys from the inputs
// (a division and a square root per splat in FP64), so the only scratch is the
// histogram and a few words of state.
//
// Exactness: x = dMSE / dMSE_MAX and m(x) are evaluated with correctly rounded
// FP64 operations in a fixed order (no contraction), the importance of each
// splat is rounded to a multiple of 2^-52 (an integer), and the budget test
// sum >= ceil(total / remaining) is on integers, so the cut cannot depend on the
// order of any summation.
#include <mutex>

#include "common.h"
#include "prune.h"

namespace potr {
namespace {

constexpr int kQBits = 52;   // importance unit 2^-52
constexpr int kPasses = 12;          // 8 digits of the key, 4 of the index
constexpr int kHistThreads = 256;
constexpr int kHistItems = 16;        // splats per thread per grid stride

// m(x) of Sec. 4.3 with the sign of a zero dropped, so that its bits order as the values.
__device__ inline double map_m(double x, double a) {
#pragma clang fp contract(off)
    double m;
    if (x >= 0.0) {
        m = x;
    } else {
        const double t = 1.0 - (2.0 * a) * x;
        m = (__builtin_sqrt(t) - 1.0) / a;
    }
    return m == 0.0 ? 0.0 : m;
}

struct Item {
    bool cand;
    bool bad;
    uint64_t key;
    int64_t q;
};

__device__ inline Item item_of(float dm, float im, double dmax, double a) {
#pragma clang fp contract(off)
    Item it;
    it.bad = !(im >= 0.f) || im > 1.f;       // NaN included
    it.cand = (double)dm < dmax;             // NaN is never a candidate
    const double x = (double)dm / dmax;
    it.key = it.cand ? (uint64_t)__double_as_longlong(map_m(x, a)) : ~0ull;
    it.q = it.bad ? 0 : (int64_t)__builtin_rint((double)im * 0x1p52);   // exact scaling by 2^52
    return it;
}

// Whether (key, index) lies in the state's region (the fixed leading bits match).
__device__ inline bool in_region(const PruneState& S, uint64_t key, uint32_t id) {
    if (S.kbits > 0 && (key >> (64 - S.kbits)) != (S.key >> (64 - S.kbits))) return false;
    if (S.ibits > 0 && (id >> (32 - S.ibits)) != (S.id >> (32 - S.ibits))) return false;
    return true;
}

__global__ void k_prune_init(PruneState* S, int64_t* hw, uint32_t* hc, int64_t* n_removed) {
    const int t = threadIdx.x;
    hw[t] = 0;
    hc[t] = 0;
    if (t == 0) {
        PruneState z{};
        *S = z;
        *n_removed = 0;
    }
}

__global__ __launch_bounds__(kHistThreads) void k_prune_hist(int64_t N, const float* __restrict__ dmse,
                                                             const float* __restrict__ imp, double dmax, double a,
                                                             int pass, PruneState* __restrict__ S,
                                                             int64_t* __restrict__ hw, uint32_t* __restrict__ hc) {
    __shared__ int64_t lw[256];
    __shared__ uint32_t lc[256];
    __shared__ int s_bad;
    const PruneState st = *S;
    if (st.done) return;
    lw[threadIdx.x] = 0;
    lc[threadIdx.x] = 0;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    const int64_t stride = (int64_t)gridDim.x * kHistThreads * kHistItems;
    bool bad = false;
    for (int64_t b0 = (int64_t)blockIdx.x * kHistThreads * kHistItems; b0 < N; b0 += stride) {
#pragma unroll 4
        for (int k = 0; k < kHistItems; ++k) {
            const int64_t i = b0 + (int64_t)k * kHistThreads + threadIdx.x;
            if (i >= N) break;
            const Item it = item_of(dmse[i], imp[i], dmax, a);
            bad = bad || it.bad;
            if (!it.cand || !in_region(st, it.key, (uint32_t)i)) continue;
            const int d = pass < 8 ? (int)((it.key >> (56 - 8 * pass)) & 255u)
                                   : (int)(((uint32_t)i >> (24 - 8 * (pass - 8))) & 255u);
            if (it.q != 0) atomicAdd((unsigned long long*)&lw[d], (unsigned long long)it.q);
            atomicAdd(&lc[d], 1u);
        }
    }
    if (bad) s_bad = 1;
    __syncthreads();
    const int d = threadIdx.x;
    if (lw[d] != 0) atomicAdd((unsigned long long*)&hw[d], (unsigned long long)lw[d]);
    if (lc[d] != 0) atomicAdd(&hc[d], lc[d]);
    if (d == 0 && s_bad) atomicOr(&S->bad, 1);
}

// One block of 256 threads: the digit where the running sum reaches the budget.
__global__ __launch_bounds__(256) void k_prune_scan(int pass, int32_t remaining, PruneState* __restrict__ S,
                                                    int64_t* __restrict__ hw, uint32_t* __restrict__ hc,
                                                    int64_t* __restrict__ n_removed) {
    __shared__ int64_t wsum[4];
    __shared__ int s_first;
    const int d = threadIdx.x, lane = d & 63, w = d >> 6;
    PruneState st = *S;
    if (st.done) return;
    const int64_t x = hw[d];
    hw[d] = 0;   // cleared for the next pass
    hc[d] = 0;
    int64_t inc = x;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const int64_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    if (d == 0) s_first = 256;
    __syncthreads();
    int64_t before = 0, all = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < w) before += wsum[k];
        all += wsum[k];
    }
    inc += before;   // inclusive prefix over the digits
    if (pass == 0) {
        // the first pass sees every candidate: its sum is the total
        if (st.bad || all > (int64_t(2) << kQBits) || all == 0) {
            if (d == 0) {
                st.done = 1;
                st.total = all;
                *S = st;
                *n_removed = st.bad || all > (int64_t(2) << kQBits) ? -1 : 0;
            }
            return;
        }
        st.total = all;
        st.need = (all + remaining - 1) / remaining;
    }
    if (st.base + inc >= st.need) atomicMin(&s_first, d);
    __syncthreads();
    if (d == s_first) {
        st.base += inc - x;
        if (pass < 8) {
            st.key |= (uint64_t)d << (56 - 8 * pass);
            st.kbits += 8;
        } else {
            st.id |= (uint32_t)d << (24 - 8 * (pass - 8));
            st.ibits += 8;
        }
        *S = st;
    }
}

__global__ __launch_bounds__(256) void k_prune_mark(int64_t N, const float* __restrict__ dmse,
                                                    const float* __restrict__ imp, double dmax, double a,
                                                    const PruneState* __restrict__ S, uint8_t* __restrict__ remove,
                                                    int64_t* __restrict__ n_removed) {
    __shared__ uint32_t cnt;
    const PruneState st = *S;
    if (threadIdx.x == 0) cnt = 0;
    __syncthreads();
    uint32_t mine = 0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < N; i += (int64_t)gridDim.x * 256) {
        bool r = false;
        if (!st.done) {
            const Item it = item_of(dmse[i], imp[i], dmax, a);
            r = it.cand && (it.key < st.key || (it.key == st.key && (uint32_t)i <= st.id));
        }
        remove[i] = r ? 1 : 0;
        mine += r ? 1u : 0u;
    }
    if (mine) atomicAdd(&cnt, mine);
    __syncthreads();
    if (threadIdx.x == 0 && cnt && !st.done) atomicAdd((unsigned long long*)n_removed, (unsigned long long)cnt);
}

// ---------------------------------------------------------------- compaction
constexpr int kCompactBlock = 1024;   // splats per block of the compaction (256 threads x 4)

__device__ inline uint32_t block_excl_scan256(uint32_t v, uint32_t* wsum, uint32_t& total) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = v;
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const uint32_t u = __shfl_up(inc, o, 64);
        if (lane >= o) inc += u;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t before = 0;
    total = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (k < w) before += wsum[k];
        total += wsum[k];
    }
    __syncthreads();
    return before + inc - v;
}

__global__ __launch_bounds__(256) void k_keep_count(int64_t N, const uint8_t* __restrict__ remove,
                                                    uint32_t* __restrict__ bcount) {
    __shared__ uint32_t wsum[4];
    const int64_t i0 = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x * 4;
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) c += (i0 + k < N && !remove[i0 + k]) ? 1u : 0u;
    uint32_t total;
    block_excl_scan256(c, wsum, total);
    if (threadIdx.x == 0) bcount[blockIdx.x] = total;
}

// Exclusive scan of the block counts in place (one block), and the survivor count.
__global__ __launch_bounds__(256) void k_keep_scan(int64_t nb, uint32_t* __restrict__ bcount,
                                                   int64_t* __restrict__ n_kept) {
    __shared__ uint32_t wsum[4];
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nb; b0 += 256) {
        const int64_t b = b0 + threadIdx.x;
        const uint32_t c = b < nb ? bcount[b] : 0u;
        uint32_t total;
        const uint32_t ex = block_excl_scan256(c, wsum, total);
        if (b < nb) bcount[b] = (uint32_t)(carry + ex);
        carry += total;
    }
    if (threadIdx.x == 0) *n_kept = carry;
}

__global__ __launch_bounds__(256) void k_keep_scatter(int64_t N, const uint8_t* __restrict__ remove,
                                                      const uint32_t* __restrict__ boff, PruneArrays in,
                                                      PruneOut out) {
    __shared__ uint32_t wsum[4];
    const int64_t i0 = (int64_t)blockIdx.x * kCompactBlock + threadIdx.x * 4;
    bool keep[4];
    uint32_t c = 0;
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        keep[k] = i0 + k < N && !remove[i0 + k];
        c += keep[k] ? 1u : 0u;
    }
    uint32_t total;
    uint32_t dst = boff[blockIdx.x] + block_excl_scan256(c, wsum, total);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
        if (!keep[k]) continue;
        const int64_t i = i0 + k;
        for (int e = 0; e < 3; ++e) {
            out.means[3 * (int64_t)dst + e] = in.means[3 * i + e];
            out.scales[3 * (int64_t)dst + e] = in.scales[3 * i + e];
        }
        reinterpret_cast<float4*>(out.quats)[dst] = reinterpret_cast<const float4*>(in.quats)[i];
        out.opac[dst] = in.opac[i];
        const float4* src = reinterpret_cast<const float4*>(in.sh + 48 * i);
        float4* to = reinterpret_cast<float4*>(out.sh + 48 * (int64_t)dst);
#pragma unroll
        for (int e = 0; e < 12; ++e) to[e] = src[e];
        out.ids[dst] = in.ids ? in.ids[i] : (int32_t)i;
        ++dst;
    }
}

int hist_grid(int64_t N) {
    const int64_t per = (int64_t)kHistThreads * kHistItems;
    const int64_t b = (N + per - 1) / per;
    return (int)(b < 1 ? 1 : (b > 2048 ? 2048 : b));
}

}  // namespace

size_t prune_select_scratch_bytes() { return sizeof(PruneState) + 256 * 8 + 256 * 4; }

potr_status launch_prune_select(int64_t N, const float* dmse, const float* imp, double dmax, int32_t remaining,
                                double a, void* scratch, uint8_t* remove, int64_t* n_removed, hipStream_t s) {
    char* p = (char*)scratch;
    PruneState* S = (PruneState*)p;
    int64_t* hw = (int64_t*)(p + sizeof(PruneState));
    uint32_t* hc = (uint32_t*)(p + sizeof(PruneState) + 256 * 8);
    hipLaunchKernelGGL(k_prune_init, dim3(1), dim3(256), 0, s, S, hw, hc, n_removed);
    potr_status st = check_launch("k_prune_init");
    if (st != POTR_OK || N == 0) return st;
    const int g = hist_grid(N);
    for (int pass = 0; pass < kPasses; ++pass) {
        hipLaunchKernelGGL(k_prune_hist, dim3(g), dim3(kHistThreads), 0, s, N, dmse, imp, dmax, a, pass, S, hw, hc);
        hipLaunchKernelGGL(k_prune_scan, dim3(1), dim3(256), 0, s, pass, remaining, S, hw, hc, n_removed);
    }
    st = check_launch("k_prune_hist / k_prune_scan");
    if (st != POTR_OK) return st;
    const int64_t mb = (N + 255) / 256;
    hipLaunchKernelGGL(k_prune_mark, dim3((unsigned)(mb < 4096 ? mb : 4096)), dim3(256), 0, s, N, dmse, imp, dmax,
                       a, S, remove, n_removed);
    return check_launch("k_prune_mark");
}

// ---------------------------------------------------------------- no-allocation form
// The select's scratch (state and histograms) as a file-scope device array: one
// copy per GPU, alive until the process ends. Host code never passes the array's
// name to a kernel (in host code it is only a stand-in for the symbol): its device
// address is looked up once per device with hipGetSymbolAddress and kept.
constexpr size_t kNoAllocScratchBytes = 4096;
static __device__ __align__(256) char scratch[kNoAllocScratchBytes];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

potr_status launch_prune_select_noalloc(int64_t N, const float* dmse, const float* imp, double dmax,
                                        int32_t remaining, double a, uint8_t* remove, int64_t* n_removed,
                                        hipStream_t s) {
    static_assert(sizeof(PruneState) + 256 * 8 + 256 * 4 <= kNoAllocScratchBytes, "select scratch fits");
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return fail(POTR_EHIP, "hipGetDevice: %s", hipGetErrorString(e));
    if (dev < 0 || dev >= kMaxDevices) return fail(POTR_EUNSUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    void* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lock(g_scratch_mu);
        if (!g_scratch_ptr[dev]) {
            e = hipGetSymbolAddress(&g_scratch_ptr[dev], HIP_SYMBOL(scratch));
            if (e != hipSuccess) {
                g_scratch_ptr[dev] = nullptr;
                return fail(POTR_EHIP, "hipGetSymbolAddress(scratch): %s", hipGetErrorString(e));
            }
        }
        ptr = g_scratch_ptr[dev];
    }
    return launch_prune_select(N, dmse, imp, dmax, remaining, a, ptr, remove, n_removed, s);
}

size_t prune_compact_scratch_bytes(int64_t N) {
    return (size_t)((N + kCompactBlock - 1) / kCompactBlock + 1) * 4;
}

potr_status launch_prune_compact(int64_t N, const uint8_t* remove, const PruneArrays& in, const PruneOut& out,
                                 void* scratch, int64_t* n_kept, hipStream_t s) {
    const int64_t nb = (N + kCompactBlock - 1) / kCompactBlock;
    uint32_t* bc = (uint32_t*)scratch;
    if (nb > 0) {
        hipLaunchKernelGGL(k_keep_count, dim3((unsigned)nb), dim3(256), 0, s, N, remove, bc);
    }
    hipLaunchKernelGGL(k_keep_scan, dim3(1), dim3(256), 0, s, nb, bc, n_kept);
    if (nb > 0) {
        hipLaunchKernelGGL(k_keep_scatter, dim3((unsigned)nb), dim3(256), 0, s, N, remove, bc, in, out);
    }
    return check_launch("k_keep_*");
}

}  // namespace potr
