// Depth ordering and tile binning (paper Sec. 3: splats composited in layers
// ordered by approximate depth), as a stable LSD radix sort.
//
// potr_bin: per view, a stable radix sort of the N depth keys (ties keep splat
//   id order) gives each splat its depth rank; a scan of tiles_touched in rank
//   order places every splat's (tile, rank) pairs, emitted in rank order.
// potr_sort: a stable radix sort of the pairs on the (view, tile) bits only. The
//   rank bits are already ordered, so the result is ordered by
//   (view, tile, depth key, splat id) -- the full key -- while only
//   ceil(log2(V * tiles)) bits are sorted instead of tile + 32 depth bits.
//
// Each radix pass is histogram -> exclusive scan of the [segment][digit][block]
// counts -> scatter. Blocks take 4096 consecutive elements; within a block the
// order is (wave, item, lane) and ranks are formed with 64-lane ballots, so the
// scatter is stable.
#include "common.h"

namespace potr {
namespace {

struct RadixGeom {
    int64_t seg_len;         // elements per segment when count == nullptr
    const int64_t* count;    // device element count (single segment) or nullptr
    int64_t cap;             // a device count above cap means overflow: sort nothing
    int32_t blocks_per_seg;
};

__device__ inline int64_t seg_n(const RadixGeom& g) {
    if (!g.count) return g.seg_len;
    const int64_t n = *g.count;
    return n > g.cap ? 0 : n;
}

template <typename K>
__device__ inline uint32_t digit_of(K k, int shift, uint32_t mask) {
    return (uint32_t)(k >> shift) & mask;
}

template <typename K>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const K* __restrict__ keys, RadixGeom g, int shift,
                                                              int bits, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[256];
    const int seg = blockIdx.y, b = blockIdx.x;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (int t = threadIdx.x; t < 256; t += kRadixThreads) h[t] = 0;
    __syncthreads();
    const int64_t n = seg_n(g);
    const K* base = keys + (int64_t)seg * g.seg_len;
#pragma unroll 4
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t e = (int64_t)b * kRadixTile + (int64_t)k * kRadixThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[digit_of(base[e], shift, mask)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < radix; d += kRadixThreads)
        hist[((int64_t)seg * radix + d) * g.blocks_per_seg + b] = h[d];
}

// Scatter one block's keys (and values) to their stable sorted positions.
// offs: exclusive scan of the histogram (global positions over all segments).
template <typename K, bool VALS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const K* __restrict__ kin, K* __restrict__ kout,
                                                                 const uint32_t* __restrict__ vin,
                                                                 uint32_t* __restrict__ vout, RadixGeom g,
                                                                 int shift, int bits,
                                                                 const uint32_t* __restrict__ offs) {
    constexpr int NW = kRadixThreads / 64;
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t goff[256];
    const int seg = blockIdx.y, b = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (int t = threadIdx.x; t < NW * 256; t += kRadixThreads) (&wcnt[0][0])[t] = 0;
    for (uint32_t d = threadIdx.x; d < radix; d += kRadixThreads)
        goff[d] = offs[((int64_t)seg * radix + d) * g.blocks_per_seg + b];
    __syncthreads();

    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.seg_len;
    const int64_t wbase = (int64_t)b * kRadixTile + (int64_t)w * (64 * kRadixItems);
    K key[kRadixItems];
    uint32_t val[kRadixItems];
    uint32_t rnk[kRadixItems];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        const int64_t e = wbase + k * 64 + lane;
        const bool ok = e < n;
        key[k] = ok ? kin[seg0 + e] : (K)0;
        if (VALS) val[k] = ok ? (vin ? vin[seg0 + e] : (uint32_t)e) : 0u;
        const uint32_t d = digit_of(key[k], shift, mask);
        uint64_t m = __ballot(ok);
        for (int bit = 0; bit < bits; ++bit) {
            const uint64_t bal = __ballot((d >> bit) & 1u);
            m &= ((d >> bit) & 1u) ? bal : ~bal;
        }
        const uint32_t below = (uint32_t)__popcll(m & lt_mask);
        const uint32_t cnt = (uint32_t)__popcll(m);
        uint32_t r = 0;
        if (ok) r = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wcnt[w][d] = r + cnt;
        __builtin_amdgcn_wave_barrier();
        rnk[k] = ok ? r + below : 0xffffffffu;
    }
    __syncthreads();
    // wave-level exclusive prefix per digit (waves hold consecutive runs)
    for (uint32_t d = threadIdx.x; d < radix; d += kRadixThreads) {
        uint32_t run = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww) {
            const uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kRadixItems; ++k) {
        if (rnk[k] == 0xffffffffu) continue;
        const uint32_t d = digit_of(key[k], shift, mask);
        const int64_t pos = (int64_t)goff[d] + wcnt[w][d] + rnk[k];
        kout[pos] = key[k];
        if (VALS) vout[pos] = val[k];
    }
}

// One LSD pass: hist -> scan -> scatter.
template <typename K, bool VALS>
potr_status radix_pass(const K* kin, K* kout, const uint32_t* vin, uint32_t* vout, const RadixGeom& g,
                       int32_t n_segs, int shift, int bits, uint32_t* hist, void* scan_tmp, hipStream_t s) {
    const dim3 grid((unsigned)g.blocks_per_seg, (unsigned)n_segs);
    hipLaunchKernelGGL(k_radix_hist<K>, grid, dim3(kRadixThreads), 0, s, kin, g, shift, bits, hist);
    potr_status st = check_launch("k_radix_hist");
    if (st != POTR_OK) return st;
    const int64_t nh = (int64_t)n_segs * (1 << bits) * g.blocks_per_seg;
    st = scan_u32(hist, hist, nh, scan_tmp, s);
    if (st != POTR_OK) return st;
    hipLaunchKernelGGL((k_radix_scatter<K, VALS>), grid, dim3(kRadixThreads), 0, s, kin, kout, vin, vout, g, shift,
                       bits, (const uint32_t*)hist);
    return check_launch("k_radix_scatter");
}

// ---------------------------------------------------------------- bin kernels
__global__ void k_depth_keys(const potr_proj* __restrict__ proj, int64_t total, uint32_t* __restrict__ keys) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    keys[i] = __float_as_uint(proj[i].depth);
}

__global__ void k_gather_counts(const uint32_t* __restrict__ order, const int32_t* __restrict__ tiles_touched,
                                int64_t N, int64_t total, int32_t* __restrict__ cnt) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    const int64_t v = i / N;
    cnt[i] = tiles_touched[v * N + order[i]];
}

__global__ void k_emit(const uint32_t* __restrict__ order, const int32_t* __restrict__ cnt,
                       const int64_t* __restrict__ offs, const potr_proj* __restrict__ proj, int64_t N,
                       int64_t total, int32_t tiles_x, int32_t tiles_per_view, int64_t capacity,
                       const int64_t* __restrict__ n_pairs, uint64_t* __restrict__ pairs) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= total) return;
    if (*n_pairs > capacity) return;
    const int32_t c = cnt[i];
    if (c == 0) return;
    const int64_t v = i / N, r = i - v * N;
    const potr_proj& p = proj[v * N + order[i]];
    int64_t o = offs[i];
    const uint64_t lo = (uint64_t)r;
    const uint64_t gbase = (uint64_t)v * (uint64_t)tiles_per_view;
    for (int ty = p.rect[1]; ty < p.rect[3]; ++ty)
        for (int tx = p.rect[0]; tx < p.rect[2]; ++tx)
            pairs[o++] = ((gbase + (uint64_t)(ty * tiles_x + tx)) << 32) | lo;
}

// ---------------------------------------------------------------- sort kernels
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_finalize(const uint64_t* __restrict__ sorted, const int64_t* __restrict__ n_pairs, int64_t cap,
                           const uint32_t* __restrict__ order, int64_t N, int32_t tiles_per_view,
                           uint32_t* __restrict__ ids, int32_t* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_pairs;
    if (n > cap) n = 0;
    if (i >= n) return;
    const uint64_t p = sorted[i];
    const uint32_t gt = (uint32_t)(p >> 32);
    const uint32_t r = (uint32_t)p;
    const uint32_t v = gt / (uint32_t)tiles_per_view;
    ids[i] = order[(int64_t)v * N + r];
    if (i == 0 || (uint32_t)(sorted[i - 1] >> 32) != gt) ranges[2 * (int64_t)gt] = (int32_t)i;
    if (i == n - 1 || (uint32_t)(sorted[i + 1] >> 32) != gt) ranges[2 * (int64_t)gt + 1] = (int32_t)(i + 1);
}

struct BinWs {
    uint32_t *ka, *kb, *va, *hist;
    int32_t* cnt;
    int64_t* offs;
    void* scan_tmp;
    size_t bytes;
};

BinWs bin_layout(int64_t N, int32_t V, char* base) {
    const int64_t VN = N * V;
    const int64_t bps = ceil_div(N > 0 ? N : 1, kRadixTile);
    BinWs w;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    w.ka = (uint32_t*)take(4 * VN);
    w.kb = (uint32_t*)take(4 * VN);
    w.va = (uint32_t*)take(4 * VN);
    w.hist = (uint32_t*)take(4 * (size_t)V * 256 * bps);
    w.cnt = (int32_t*)take(4 * VN);
    w.offs = (int64_t*)take(8 * VN);
    const int64_t ns = VN > (int64_t)V * 256 * bps ? VN : (int64_t)V * 256 * bps;
    w.scan_tmp = take(scan_tmp_bytes(ns));
    w.bytes = o;
    return w;
}

struct SortWs {
    uint64_t* alt;
    uint32_t* hist;
    void* scan_tmp;
    size_t bytes;
};

SortWs sort_layout(int64_t cap, char* base) {
    const int64_t nb = ceil_div(cap > 0 ? cap : 1, kRadixTile);
    SortWs w;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    w.alt = (uint64_t*)take(8 * (size_t)(cap > 0 ? cap : 1));
    w.hist = (uint32_t*)take(4 * (size_t)256 * nb);
    w.scan_tmp = take(scan_tmp_bytes(256 * nb));
    w.bytes = o;
    return w;
}

}  // namespace

size_t bin_workspace_bytes(int64_t N, int32_t V) { return bin_layout(N, V, nullptr).bytes; }

potr_status launch_bin(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                       const potr_proj* proj, const int32_t* tiles_touched, void* ws, uint32_t* order,
                       uint64_t* pairs, int64_t capacity, int64_t* n_pairs, hipStream_t s) {
    BinWs w = bin_layout(N, V, (char*)ws);
    const int64_t VN = N * V;
    const int txs = tiles_x(cam0, cfg), tpv = txs * tiles_y(cam0, cfg);
    if (VN == 0) return scan_i32_to_i64(nullptr, nullptr, 0, n_pairs, w.scan_tmp, s);
    const unsigned gb = (unsigned)ceil_div(VN, 256);
    hipLaunchKernelGGL(k_depth_keys, dim3(gb), dim3(256), 0, s, proj, VN, w.ka);
    potr_status st = check_launch("k_depth_keys");
    if (st != POTR_OK) return st;
    // stable per-view sort of the 32-bit depth keys; four 8-bit passes
    RadixGeom g{N, nullptr, 0, (int32_t)ceil_div(N, kRadixTile)};
    uint32_t *kin = w.ka, *kout = w.kb, *vin = nullptr, *vout = w.va;
    for (int pass = 0; pass < 4; ++pass) {
        if (pass == 3) vout = order;
        st = radix_pass<uint32_t, true>(kin, kout, vin, vout, g, V, 8 * pass, 8, w.hist, w.scan_tmp, s);
        if (st != POTR_OK) return st;
        uint32_t* t = kin; kin = kout; kout = t;
        vin = vout;
        vout = (vout == w.va) ? order : w.va;
    }
    hipLaunchKernelGGL(k_gather_counts, dim3(gb), dim3(256), 0, s, (const uint32_t*)order, tiles_touched, N, VN,
                       w.cnt);
    st = check_launch("k_gather_counts");
    if (st != POTR_OK) return st;
    st = scan_i32_to_i64(w.cnt, w.offs, VN, n_pairs, w.scan_tmp, s);
    if (st != POTR_OK) return st;
    hipLaunchKernelGGL(k_emit, dim3(gb), dim3(256), 0, s, (const uint32_t*)order, (const int32_t*)w.cnt,
                       (const int64_t*)w.offs, proj, N, VN, txs, tpv, capacity, (const int64_t*)n_pairs, pairs);
    return check_launch("k_emit");
}

size_t sort_workspace_bytes(int64_t capacity, int32_t, int32_t) { return sort_layout(capacity, nullptr).bytes; }

potr_status launch_sort(int64_t N, int32_t V, int32_t tiles_per_view, const int64_t* n_pairs, int64_t n_max,
                        uint64_t* pairs, const uint32_t* order, void* ws, uint32_t* sorted_ids,
                        int32_t* tile_ranges, hipStream_t s) {
    SortWs w = sort_layout(n_max, (char*)ws);
    const int64_t ranges_n = 2 * (int64_t)V * tiles_per_view;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(ranges_n, 256)), dim3(256), 0, s, tile_ranges, ranges_n, 0);
    potr_status st = check_launch("k_fill_i32");
    if (st != POTR_OK || n_max == 0) return st;
    int bits = 1;
    while ((int64_t(1) << bits) < (int64_t)V * tiles_per_view) ++bits;
    const int passes = (bits + 7) / 8;
    const int per = (bits + passes - 1) / passes;
    RadixGeom g{0, n_pairs, n_max, (int32_t)ceil_div(n_max, kRadixTile)};
    uint64_t *kin = pairs, *kout = w.alt;
    for (int p = 0; p < passes; ++p) {
        const int b = (p == passes - 1) ? bits - per * p : per;
        st = radix_pass<uint64_t, false>(kin, kout, nullptr, nullptr, g, 1, 32 + per * p, b, w.hist, w.scan_tmp, s);
        if (st != POTR_OK) return st;
        uint64_t* t = kin; kin = kout; kout = t;
    }
    hipLaunchKernelGGL(k_finalize, dim3((unsigned)ceil_div(n_max, 256)), dim3(256), 0, s, (const uint64_t*)kin,
                       n_pairs, n_max, order, N, tiles_per_view, sorted_ids, tile_ranges);
    return check_launch("k_finalize");
}

}  // namespace potr
