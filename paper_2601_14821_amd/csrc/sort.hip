// Depth ordering and tile binning (paper Sec. 3: splats composited in layers
// ordered by approximate depth), as a stable LSD radix sort.
//
// potr_bin: per view, a stable radix sort of the N depth keys (ties keep splat
//   id order) gives each splat its depth rank; a scan of tiles_touched in rank
//   order places every splat's (tile, rank) pairs, emitted in rank order.
// potr_sort: a stable radix sort of the pairs on the (view, tile) bits only.
//   Pairs were emitted in depth-rank order and the sort is stable, so the
//   result is ordered by (view, tile, depth key, splat id) -- the full key --
//   while only ceil(log2(V * tiles)) bits are sorted instead of tile + 32 depth
//   bits. The low bits carry the splat id as payload.
//
// Pairs are packed as ((view * tiles + tile) << id_bits) | splat id in 32 bits
// when both fields fit, else in 64 bits with the id in the low word.
//
// Each radix pass is histogram -> exclusive scan of the [segment][digit][block]
// counts -> scatter. Blocks take ITEMS x 256 consecutive elements; within a
// block the order is (wave, item, lane) and ranks come from 64-lane ballots, so
// the scatter is stable. Each block first sorts its elements in LDS, then
// writes every digit's run to consecutive addresses.
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

template <typename K, int ITEMS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_hist(const K* __restrict__ keys, RadixGeom g, int shift,
                                                              int bits, uint32_t* __restrict__ hist) {
    constexpr int TILE = kRadixThreads * ITEMS;
    __shared__ uint32_t h[256];
    const int seg = blockIdx.y, b = blockIdx.x;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (int t = threadIdx.x; t < 256; t += kRadixThreads) h[t] = 0;
    __syncthreads();
    const int64_t n = seg_n(g);
    const K* base = keys + (int64_t)seg * g.seg_len;
#pragma unroll 4
    for (int k = 0; k < ITEMS; ++k) {
        const int64_t e = (int64_t)b * TILE + (int64_t)k * kRadixThreads + threadIdx.x;
        if (e < n) atomicAdd(&h[digit_of(base[e], shift, mask)], 1u);
    }
    __syncthreads();
    for (uint32_t d = threadIdx.x; d < radix; d += kRadixThreads)
        hist[((int64_t)seg * radix + d) * g.blocks_per_seg + b] = h[d];
}

// Scatter one block's keys (and values) to their stable sorted positions.
// offs: exclusive scan of the histogram (global positions over all segments).
template <typename K, bool VALS, int ITEMS>
__global__ __launch_bounds__(kRadixThreads) void k_radix_scatter(const K* __restrict__ kin, K* __restrict__ kout,
                                                                 const uint32_t* __restrict__ vin,
                                                                 uint32_t* __restrict__ vout, RadixGeom g,
                                                                 int shift, int bits,
                                                                 const uint32_t* __restrict__ offs) {
    constexpr int NW = kRadixThreads / 64;
    constexpr int TILE = kRadixThreads * ITEMS;
    __shared__ uint32_t wcnt[NW][256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t boff[256];
    __shared__ uint32_t wsum[NW];
    __shared__ K s_key[TILE];
    __shared__ uint32_t s_val[VALS ? TILE : 1];
    const int seg = blockIdx.y, b = blockIdx.x;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t radix = 1u << bits, mask = radix - 1;
    for (int t = threadIdx.x; t < NW * 256; t += kRadixThreads) (&wcnt[0][0])[t] = 0;
    for (uint32_t d = threadIdx.x; d < radix; d += kRadixThreads)
        goff[d] = offs[((int64_t)seg * radix + d) * g.blocks_per_seg + b];
    __syncthreads();

    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.seg_len;
    const int64_t blk0 = (int64_t)b * TILE;
    const int64_t wbase = blk0 + (int64_t)w * (64 * ITEMS);
    K key[ITEMS];
    uint32_t val[ITEMS];
    uint32_t rnk[ITEMS];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
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
    // per digit: exclusive prefix over waves (waves hold consecutive runs) and the block total
    for (uint32_t d = threadIdx.x; d < 256; d += kRadixThreads) {
        uint32_t run = 0;
        if (d < radix) {
#pragma unroll
            for (int ww = 0; ww < NW; ++ww) {
                const uint32_t c = wcnt[ww][d];
                wcnt[ww][d] = run;
                run += c;
            }
        }
        boff[d] = run;
    }
    __syncthreads();
    // exclusive scan of the block's digit totals (256 entries, one per thread)
    {
        const uint32_t x = boff[threadIdx.x];
        uint32_t inc = x;
#pragma unroll
        for (int dd = 1; dd < 64; dd <<= 1) {
            const uint32_t y = __shfl_up(inc, dd, 64);
            if (lane >= dd) inc += y;
        }
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0;
#pragma unroll
        for (int ww = 0; ww < NW; ++ww)
            if (ww < w) pre += wsum[ww];
        boff[threadIdx.x] = pre + inc - x;
    }
    __syncthreads();
    // block-local sort in LDS
#pragma unroll
    for (int k = 0; k < ITEMS; ++k) {
        if (rnk[k] == 0xffffffffu) continue;
        const uint32_t d = digit_of(key[k], shift, mask);
        const uint32_t p = boff[d] + wcnt[w][d] + rnk[k];
        s_key[p] = key[k];
        if (VALS) s_val[p] = val[k];
    }
    __syncthreads();
    // coalesced write-out: digit runs go to consecutive global addresses
    const int64_t left = n - blk0;
    const int cnt_blk = left < TILE ? (int)(left > 0 ? left : 0) : TILE;
    for (int i = threadIdx.x; i < cnt_blk; i += kRadixThreads) {
        const K kk = s_key[i];
        const uint32_t d = digit_of(kk, shift, mask);
        const int64_t pos = (int64_t)goff[d] + (i - (int)boff[d]);
        kout[pos] = kk;
        if (VALS) vout[pos] = s_val[i];
    }
}

template <typename K, bool VALS, int ITEMS>
potr_status radix_pass(const K* kin, K* kout, const uint32_t* vin, uint32_t* vout, const RadixGeom& g,
                       int32_t n_segs, int shift, int bits, uint32_t* hist, void* scan_tmp, hipStream_t s) {
    const dim3 grid((unsigned)g.blocks_per_seg, (unsigned)n_segs);
    hipLaunchKernelGGL((k_radix_hist<K, ITEMS>), grid, dim3(kRadixThreads), 0, s, kin, g, shift, bits, hist);
    potr_status st = check_launch("k_radix_hist");
    if (st != POTR_OK) return st;
    const int64_t nh = (int64_t)n_segs * (1 << bits) * g.blocks_per_seg;
    st = scan_u32(hist, hist, nh, scan_tmp, s);
    if (st != POTR_OK) return st;
    hipLaunchKernelGGL((k_radix_scatter<K, VALS, ITEMS>), grid, dim3(kRadixThreads), 0, s, kin, kout, vin, vout, g,
                       shift, bits, (const uint32_t*)hist);
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

// Pairs of 256 consecutive (view, rank) entries, written cooperatively by the
// block so that stores are contiguous: each output slot finds its splat by a
// binary search over the block's offsets.
template <typename K>
__global__ __launch_bounds__(256) void k_emit(const uint32_t* __restrict__ order, const int32_t* __restrict__ cnt,
                                              const int64_t* __restrict__ offs, const potr_proj* __restrict__ proj,
                                              int64_t N, int64_t total, int32_t tiles_x, int32_t tiles_per_view,
                                              int rank_bits, int64_t capacity, const int64_t* __restrict__ n_pairs,
                                              K* __restrict__ pairs) {
    __shared__ int64_t s_off[256];
    __shared__ uint32_t s_key0[256];      // (view * tiles + y0 * tiles_x + x0)
    __shared__ uint32_t s_sid[256];       // splat id
    __shared__ uint16_t s_w[256];
    if (*n_pairs > capacity) return;
    const int64_t i0 = (int64_t)blockIdx.x * 256;
    const int64_t i = i0 + threadIdx.x;
    int64_t my_off = 0;
    if (i < total) {
        const int64_t v = i / N;
        const int32_t c = cnt[i];
        my_off = offs[i];
        const uint32_t id = order[i];
        const potr_proj& p = proj[v * N + id];
        s_key0[threadIdx.x] = (uint32_t)(v * tiles_per_view + p.rect[1] * tiles_x + p.rect[0]);
        s_sid[threadIdx.x] = id;
        s_w[threadIdx.x] = (uint16_t)(c > 0 ? p.rect[2] - p.rect[0] : 1);
    } else {
        s_key0[threadIdx.x] = 0;
        s_sid[threadIdx.x] = 0;
        s_w[threadIdx.x] = 1;
    }
    s_off[threadIdx.x] = my_off;
    __syncthreads();
    const int64_t last = (total - i0 < 256 ? total - i0 : 256) - 1;
    const int64_t beg = s_off[0];
    const int64_t end = offs[i0 + last] + cnt[i0 + last];
    for (int64_t p = beg + threadIdx.x; p < end; p += 256) {
        int lo = 0, hi = (int)last;          // last entry with s_off <= p
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (s_off[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        const uint32_t t = (uint32_t)(p - s_off[lo]);
        const uint32_t wdt = s_w[lo];
        const uint32_t ty = t / wdt, tx = t - ty * wdt;
        const uint64_t g = (uint64_t)s_key0[lo] + (uint64_t)ty * (uint32_t)tiles_x + tx;
        if (sizeof(K) == 4)
            pairs[p] = (K)((g << rank_bits) | s_sid[lo]);
        else
            pairs[p] = (K)((g << 32) | s_sid[lo]);
    }
}

// ---------------------------------------------------------------- sort kernels
__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

template <typename K>
__global__ void k_finalize(const K* __restrict__ sorted, const int64_t* __restrict__ n_pairs, int64_t cap,
                           int rank_bits, uint32_t* __restrict__ ids, int32_t* __restrict__ ranges) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t n = *n_pairs;
    if (n > cap) n = 0;
    if (i >= n) return;
    const int sh = sizeof(K) == 4 ? rank_bits : 32;
    const uint64_t rmask = sizeof(K) == 4 ? ((1ull << rank_bits) - 1) : 0xffffffffull;
    const K p = sorted[i];
    const uint32_t gt = (uint32_t)((uint64_t)p >> sh);
    ids[i] = (uint32_t)((uint64_t)p & rmask);
    if (i == 0 || (uint32_t)((uint64_t)sorted[i - 1] >> sh) != gt) ranges[2 * (int64_t)gt] = (int32_t)i;
    if (i == n - 1 || (uint32_t)((uint64_t)sorted[i + 1] >> sh) != gt) ranges[2 * (int64_t)gt + 1] = (int32_t)(i + 1);
}

constexpr int kDepthItems = 4;       // depth sort: 1024 keys per block (N-sized, fills the GPU)
constexpr int kPairItems = kRadixItems;

int bit_width(int64_t x) {           // bits to hold 0..x (at least 1)
    int b = 1;
    while (b < 62 && (int64_t(1) << b) <= x) ++b;
    return b;
}

struct Packing {
    int tile_bits, rank_bits;
    bool u32;
};

Packing packing(int64_t N, int32_t V, int32_t tiles_per_view) {
    Packing p;
    p.tile_bits = bit_width((int64_t)V * tiles_per_view - 1);
    p.rank_bits = bit_width(N > 0 ? N - 1 : 0);
    p.u32 = p.tile_bits + p.rank_bits <= 32;
    return p;
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
    const int64_t bps = ceil_div(N > 0 ? N : 1, kRadixThreads * kDepthItems);
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
    void* alt;
    uint32_t* hist;
    void* scan_tmp;
    size_t bytes;
};

SortWs sort_layout(int64_t cap, char* base) {
    const int64_t nb = ceil_div(cap > 0 ? cap : 1, kRadixThreads * kPairItems);
    SortWs w;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    w.alt = take(8 * (size_t)(cap > 0 ? cap : 1));
    w.hist = (uint32_t*)take(4 * (size_t)256 * nb);
    w.scan_tmp = take(scan_tmp_bytes(256 * nb));
    w.bytes = o;
    return w;
}

template <typename K>
potr_status emit_pairs(const uint32_t* order, const BinWs& w, const potr_proj* proj, int64_t N, int64_t VN,
                       int txs, int tpv, int rank_bits, int64_t capacity, const int64_t* n_pairs, void* pairs,
                       hipStream_t s) {
    hipLaunchKernelGGL(k_emit<K>, dim3((unsigned)ceil_div(VN, 256)), dim3(256), 0, s, order, (const int32_t*)w.cnt,
                       (const int64_t*)w.offs, proj, N, VN, txs, tpv, rank_bits, capacity, n_pairs, (K*)pairs);
    return check_launch("k_emit");
}

template <typename K>
potr_status sort_pairs(int64_t N, int32_t V, int32_t tpv, const Packing& pk, const int64_t* n_pairs, int64_t n_max,
                       void* pairs, const SortWs& w, uint32_t* sorted_ids,
                       int32_t* tile_ranges, hipStream_t s) {
    const int bits = pk.tile_bits;
    const int passes = (bits + 7) / 8;
    const int per = (bits + passes - 1) / passes;
    const int shift0 = sizeof(K) == 4 ? pk.rank_bits : 32;
    RadixGeom g{0, n_pairs, n_max, (int32_t)ceil_div(n_max, kRadixThreads * kPairItems)};
    K *kin = (K*)pairs, *kout = (K*)w.alt;
    for (int p = 0; p < passes; ++p) {
        const int b = (p == passes - 1) ? bits - per * p : per;
        potr_status st = radix_pass<K, false, kPairItems>(kin, kout, nullptr, nullptr, g, 1, shift0 + per * p, b,
                                                          w.hist, w.scan_tmp, s);
        if (st != POTR_OK) return st;
        K* t = kin; kin = kout; kout = t;
    }
    hipLaunchKernelGGL(k_finalize<K>, dim3((unsigned)ceil_div(n_max, 256)), dim3(256), 0, s, (const K*)kin, n_pairs,
                       n_max, pk.rank_bits, sorted_ids, tile_ranges);
    return check_launch("k_finalize");
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
    RadixGeom g{N, nullptr, 0, (int32_t)ceil_div(N, kRadixThreads * kDepthItems)};
    uint32_t *kin = w.ka, *kout = w.kb, *vin = nullptr, *vout = w.va;
    for (int pass = 0; pass < 4; ++pass) {
        if (pass == 3) vout = order;
        st = radix_pass<uint32_t, true, kDepthItems>(kin, kout, vin, vout, g, V, 8 * pass, 8, w.hist, w.scan_tmp, s);
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
    const Packing pk = packing(N, V, tpv);
    if (pk.u32)
        return emit_pairs<uint32_t>(order, w, proj, N, VN, txs, tpv, pk.rank_bits, capacity, n_pairs, pairs, s);
    return emit_pairs<uint64_t>(order, w, proj, N, VN, txs, tpv, pk.rank_bits, capacity, n_pairs, pairs, s);
}

size_t sort_workspace_bytes(int64_t capacity, int32_t, int32_t) { return sort_layout(capacity, nullptr).bytes; }

potr_status launch_sort(int64_t N, int32_t V, int32_t tiles_per_view, const int64_t* n_pairs, int64_t n_max,
                        uint64_t* pairs, void* ws, uint32_t* sorted_ids, int32_t* tile_ranges, hipStream_t s) {
    SortWs w = sort_layout(n_max, (char*)ws);
    const int64_t ranges_n = 2 * (int64_t)V * tiles_per_view;
    hipLaunchKernelGGL(k_fill_i32, dim3((unsigned)ceil_div(ranges_n, 256)), dim3(256), 0, s, tile_ranges, ranges_n, 0);
    potr_status st = check_launch("k_fill_i32");
    if (st != POTR_OK || n_max == 0) return st;
    const Packing pk = packing(N, V, tiles_per_view);
    if (pk.u32)
        return sort_pairs<uint32_t>(N, V, tiles_per_view, pk, n_pairs, n_max, pairs, w, sorted_ids,
                                    tile_ranges, s);
    return sort_pairs<uint64_t>(N, V, tiles_per_view, pk, n_pairs, n_max, pairs, w, sorted_ids, tile_ranges,
                                s);
}

}  // namespace potr
