// Depth ordering and tile binning (paper Sec. 3: splats composited in layers
// ordered by approximate depth).
//
// potr_bin orders each view's splats by depth key (a stable LSD radix sort of
// the N 32-bit keys, so ties keep splat id order) and counts, for every group
// of 4096 consecutive depth ranks, the pairs its splats make in every tile and
// every tile row; from those counts come every tile's start and the number of
// pairs. potr_sort places every (tile, splat) pair (see the pair placement
// section below) so that each tile's list is in (depth key, splat id) order,
// the order a sort of (tile, depth, id) keys would give, without sorting per
// pair.
//
// Every depth radix pass is three wait-free kernels: per block of 4096 keys
// its digit counts (also summed into the view's digit totals); per (view,
// digit) a scan of those over the blocks (the blocks' first places); per block
// a stable rank of its keys by digit (ballots per wave), an LDS sort and
// coalesced runs out. The passes sort by key - min over the view's keys: a
// view whose keys span fewer than 2^24 (2^16, 2^8) values needs three (two,
// one) passes, and the rest return at once. The key range comes from one read
// up front (or from the projection that wrote the keys). No kernel waits on
// another block, so the passes share the chip with kernels on other streams
// without spinning.
#include <algorithm>

#include "common.h"
#include "dpp.h"

namespace potr {
namespace {

constexpr int kSwThreads = 1024;              // depth radix pass: 16 waves x 4 keys per lane
constexpr int kSwItems = 4;
constexpr int kSwWaves = kSwThreads / 64;
constexpr int kTile = kSwThreads * kSwItems;  // keys per block
constexpr int kMaxPasses = 4;

// Lanes of the wave (among those with ok set) whose BITS-bit key d equals this
// lane's: how many there are (cnt) and how many sit below this lane (below).
// Per bit, the bit spread over the word (0 or all ones), its ballot, and a
// mask update that keeps the lanes whose bit agrees: m &= ~(ballot ^ spread).
template <int BITS>
__device__ inline void match_rank(uint32_t d, bool ok, uint32_t& below, uint32_t& cnt) {
    const uint64_t okb = __ballot(ok);
    uint32_t mlo = (uint32_t)okb, mhi = (uint32_t)(okb >> 32);
#pragma unroll
    for (int bit = 0; bit < BITS; ++bit) {
        const uint32_t r = (uint32_t)((int32_t)(d << (31 - bit)) >> 31);
        const uint64_t bal = __ballot(r != 0u);
        mlo &= ~((uint32_t)bal ^ r);
        mhi &= ~((uint32_t)(bal >> 32) ^ r);
    }
    below = __builtin_amdgcn_mbcnt_hi(mhi, __builtin_amdgcn_mbcnt_lo(mlo, 0u));
    cnt = (uint32_t)(__popc(mlo) + __popc(mhi));
}

// Exclusive scan of one value per thread over the block (NT threads).
template <int NT>
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t inc = wave_incl_scan(x);
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int k = 0; k < NT / 64; ++k)
        if (k < w) pre += wsum[k];
    __syncthreads();
    return pre + inc - x;
}

template <typename K>
__device__ inline uint32_t digit_of(K k, int shift, uint32_t mask) {
    return (uint32_t)(k >> shift) & mask;
}

// ---------------------------------------------------------------- pass geometry
struct Seg {
    int64_t len;             // elements per segment when count == nullptr
    const int64_t* count;    // device element count (single segment) or nullptr
    int64_t cap;             // a device count outside [0, cap] means: sort nothing
    int32_t bps;             // blocks per segment
};

__device__ inline int64_t seg_n(const Seg& g) {
    if (!g.count) return g.len;
    const int64_t n = *g.count;
    return (n < 0 || n > g.cap) ? 0 : n;
}

struct Pass {
    int32_t pass, shift, bits;
    uint32_t* ghist;          // this pass's digit totals at ghist[seg * kMaxPasses * 256 + digit] (cleared, then summed by k_pass_count)
    uint32_t* offs;           // [seg][digit][block]: the block's count, then its first place for the digit
};

// Depth keys, rects and the range of the keys, per view, in one read of the
// records (the depth and the rect sit in the same 16 bytes of a record). The
// keys go to keys_out, the rects to rect_out, packed as the two words
// (x0 | x1 << 16, y0 | y1 << 16) for tiles [x0, x1) x [y0, y1); krange[v] gets
// the largest key and the largest complemented key (so the smallest key is its
// complement, and the cleared words are the identity of both maxima).
constexpr int kHistThreads = 256;
constexpr int kHistItems = 8;

__global__ __launch_bounds__(kHistThreads) void k_keys(const potr_proj* __restrict__ proj, int64_t N,
                                                      uint32_t* __restrict__ keys_out, uint2* __restrict__ rect_out,
                                                      uint32_t* __restrict__ krange) {
    __shared__ uint32_t s_hi, s_lo;
    if (threadIdx.x == 0) s_hi = s_lo = 0u;
    __syncthreads();
    const int v = blockIdx.y;
    const int64_t base = (int64_t)v * N;
    const int64_t e0 = (int64_t)blockIdx.x * (kHistThreads * kHistItems) + threadIdx.x;
    // all loads first, without branches (slots past the end load the last record)
    uint4 q[kHistItems];
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        const int64_t e = min(e0 + (int64_t)k * kHistThreads, N - 1);
        q[k] = reinterpret_cast<const uint4*>(proj + base + e)[2];   // rgb[2], depth, rect
    }
    uint32_t hi = 0u, lo = 0u;   // largest key, largest complemented key
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) {
        const int64_t e = e0 + (int64_t)k * kHistThreads;
        if (e < N) {
            const uint32_t key = q[k].y;
            keys_out[base + e] = key;
            rect_out[base + e] = make_uint2((q[k].z & 0xffffu) | (q[k].w << 16), (q[k].z >> 16) | (q[k].w & 0xffff0000u));
            hi = max(hi, key);
            lo = max(lo, ~key);
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, m, 64));
        lo = max(lo, (uint32_t)__shfl_xor((int)lo, m, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&s_hi, hi);
        atomicMax(&s_lo, lo);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(krange + 2 * v, s_hi);
        atomicMax(krange + 2 * v + 1, s_lo);
    }
}

// The key range of every view from the per-wave partials a projection launch
// left (largest key, largest complemented key per wave of 64 splats; see
// BinKeys): a grid of (blocks, view), each folding a stride of the partials.
__global__ __launch_bounds__(kHistThreads) void k_krange(const uint2* __restrict__ part, int64_t per_view,
                                                        uint32_t* __restrict__ krange) {
    __shared__ uint32_t s_hi, s_lo;
    if (threadIdx.x == 0) s_hi = s_lo = 0u;
    __syncthreads();
    const int v = blockIdx.y;
    uint32_t hi = 0u, lo = 0u;
    for (int64_t k = (int64_t)blockIdx.x * kHistThreads + threadIdx.x; k < per_view;
         k += (int64_t)gridDim.x * kHistThreads) {
        const uint2 q = part[(int64_t)v * per_view + k];
        hi = max(hi, q.x);
        lo = max(lo, q.y);
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) {
        hi = max(hi, (uint32_t)__shfl_xor((int)hi, m, 64));
        lo = max(lo, (uint32_t)__shfl_xor((int)lo, m, 64));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&s_hi, hi);
        atomicMax(&s_lo, lo);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        atomicMax(krange + 2 * v, s_hi);
        atomicMax(krange + 2 * v + 1, s_lo);
    }
}

// Radix passes needed for the offsets key - min of one view: 8 bits each, at
// least one (which then also writes the identity order of equal keys).
__device__ inline int passes_of(const uint32_t* krange, int v, uint32_t& kmin) {
    const uint32_t hi = krange[2 * v];
    kmin = ~krange[2 * v + 1];
    const uint32_t span = hi >= kmin ? hi - kmin : 0u;
    const int bits = span ? 32 - __clz((int)span) : 0;
    return max(1, (bits + 7) / 8);
}

// One stable radix pass over the depth keys of every view, by the digits of
// key - min, in three wait-free kernels (the view's passes_of decides how many
// passes it needs; the later ones return at once):
//   k_pass_count   per block of kTile keys, its count of every digit, also
//                  added into the view's totals of the digit;
//   k_pass_scan    per (view, digit), the blocks' first places for the digit
//                  (the digit's base over the view, plus the counts of the
//                  blocks before), in place of the counts;
//   k_pass_scatter per block, each key's rank among the block's keys of its
//                  digit (ballots per wave, in (wave, item, lane) order, which
//                  is the keys' order), an LDS sort of the block, and every
//                  digit's run written to consecutive addresses.
// Values come from vin, or are the element's index when vin == nullptr. A view's
// last pass writes only the values, to vfinal; the others write keys to kout and
// values to vout.
constexpr int kPcItems = 16;   // keys per thread of the count kernel (256 threads: one tile)
static_assert(256 * kPcItems == kTile, "the count kernel covers one scatter block");

__global__ __launch_bounds__(256) void k_pass_count(const uint32_t* __restrict__ kin, Seg g, Pass P,
                                                   const uint32_t* __restrict__ krange) {
    __shared__ uint32_t h[256];
    const int b = blockIdx.x, seg = blockIdx.y;
    uint32_t kmin;
    if (P.pass >= passes_of(krange, seg, kmin)) return;
    h[threadIdx.x] = 0u;
    __syncthreads();
    const int64_t n = seg_n(g), seg0 = (int64_t)seg * g.len, blk0 = (int64_t)b * kTile;
    const uint32_t mask = (1u << P.bits) - 1u;
    uint32_t key[kPcItems];
#pragma unroll
    for (int k = 0; k < kPcItems; ++k) {
        const int64_t e = blk0 + k * 256 + threadIdx.x;
        key[k] = e < n ? kin[seg0 + e] : 0u;
    }
#pragma unroll
    for (int k = 0; k < kPcItems; ++k)
        if (blk0 + k * 256 + threadIdx.x < n) atomicAdd(&h[digit_of(key[k] - kmin, P.shift, mask)], 1u);
    __syncthreads();
    const uint32_t c = h[threadIdx.x];
    P.offs[((int64_t)seg * 256 + threadIdx.x) * g.bps + b] = c;
    if (c) atomicAdd(P.ghist + (int64_t)seg * kMaxPasses * 256 + threadIdx.x, c);   // the view's digit totals
}

__global__ __launch_bounds__(256) void k_pass_scan(Seg g, Pass P, const uint32_t* __restrict__ krange) {
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t s_base;
    const int d = blockIdx.x, seg = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t kmin;
    if (P.pass >= passes_of(krange, seg, kmin)) return;
    // the digit's base: the view's keys of the digits below it
    const uint32_t gh = P.ghist[(int64_t)seg * kMaxPasses * 256 + threadIdx.x];
    const uint32_t base = block_excl_scan<256>(gh, wsum);
    if ((int)threadIdx.x == d) s_base = base;
    __syncthreads();
    uint32_t carry = s_base;
    uint32_t* row = P.offs + ((int64_t)seg * 256 + d) * g.bps;
    for (int b0 = 0; b0 < g.bps; b0 += 256) {
        const int b = b0 + (int)threadIdx.x;
        const uint32_t c = b < g.bps ? row[b] : 0u;
        const uint32_t inc = wave_incl_scan(c);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = carry, all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) pre += wsum[k];
            all += wsum[k];
        }
        if (b < g.bps) row[b] = pre + inc - c;
        carry += all;
        __syncthreads();
    }
}

__global__ __launch_bounds__(kSwThreads) void k_pass_scatter(const uint32_t* __restrict__ kin,
                                                            uint32_t* __restrict__ kout,
                                                            const uint32_t* __restrict__ vin,
                                                            uint32_t* __restrict__ vout,
                                                            uint32_t* __restrict__ vfinal, Seg g, Pass P,
                                                            const uint32_t* __restrict__ krange) {
    __shared__ uint32_t wcnt[kSwWaves][256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t boff[256];
    __shared__ uint32_t wsum[kSwWaves];
    __shared__ uint32_t s_key[kTile];
    __shared__ uint32_t s_val[kTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int b = blockIdx.x, seg = blockIdx.y;
    const uint32_t radix = 1u << P.bits, mask = radix - 1;
    uint32_t kmin;
    const int np = passes_of(krange, seg, kmin);
    if (P.pass >= np) return;   // every block of this view returns
    for (int t = threadIdx.x; t < kSwWaves * 256; t += kSwThreads) (&wcnt[0][0])[t] = 0;
    if (threadIdx.x < radix) goff[threadIdx.x] = P.offs[((int64_t)seg * 256 + threadIdx.x) * g.bps + b];
    __syncthreads();
    const bool last = P.pass == np - 1;
    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.len;
    const int64_t blk0 = (int64_t)b * kTile;
    const int64_t wbase = blk0 + (int64_t)w * (64 * kSwItems);

    uint32_t key[kSwItems];
    uint32_t val[kSwItems];
    uint32_t rnk[kSwItems];
    // all loads first and without branches (slots past the end load the last
    // element and are not used), so that they are in flight together
#pragma unroll
    for (int k = 0; k < kSwItems; ++k) {
        const int64_t e = max((int64_t)0, min(wbase + k * 64 + lane, n - 1));
        key[k] = kin[seg0 + e];
        val[k] = vin ? vin[seg0 + e] : (uint32_t)e;
    }
#pragma unroll
    for (int k = 0; k < kSwItems; ++k) {
        const int64_t e = wbase + k * 64 + lane;
        const bool ok = e < n;
        const uint32_t d = digit_of(key[k] - kmin, P.shift, mask);
        uint32_t below, cnt;
        match_rank<8>(d, ok, below, cnt);
        uint32_t r = 0;
        if (ok) r = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (ok && below == 0) wcnt[w][d] = r + cnt;
        __builtin_amdgcn_wave_barrier();
        rnk[k] = ok ? r + below : 0xffffffffu;
    }
    __syncthreads();
    // per digit: exclusive prefix over waves (waves hold consecutive runs) and the block count
    uint32_t run = 0;
    if (threadIdx.x < radix) {
        const uint32_t d = threadIdx.x;
#pragma unroll
        for (int ww = 0; ww < kSwWaves; ++ww) {
            const uint32_t c = wcnt[ww][d];
            wcnt[ww][d] = run;
            run += c;
        }
    }
    // exclusive scan of the block's digit counts: LDS position of each digit's run
    const uint32_t bo = block_excl_scan<kSwThreads>(run, wsum);
    if (threadIdx.x < 256) boff[threadIdx.x] = bo;
    __syncthreads();
    // block-local sort in LDS
#pragma unroll
    for (int k = 0; k < kSwItems; ++k) {
        if (rnk[k] == 0xffffffffu) continue;
        const uint32_t d = digit_of(key[k] - kmin, P.shift, mask);
        const uint32_t p = boff[d] + wcnt[w][d] + rnk[k];
        s_key[p] = key[k];
        s_val[p] = val[k];
    }
    __syncthreads();
    // coalesced write-out: digit runs go to consecutive global addresses
    const int64_t left = n - blk0;
    const int cnt_blk = left < kTile ? (int)(left > 0 ? left : 0) : kTile;
    for (int i = threadIdx.x; i < cnt_blk; i += kSwThreads) {
        const uint32_t kk = s_key[i];
        const uint32_t d = digit_of(kk - kmin, P.shift, mask);
        const int64_t pos = seg0 + (int64_t)goff[d] + (i - (int)boff[d]);
        if (last) {
            vfinal[pos] = s_val[i];
        } else {
            kout[pos] = kk;
            vout[pos] = s_val[i];
        }
    }
}

// Clears 64-bit words (digit totals, key range, tickets).
__global__ void k_clear(uint64_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// ---------------------------------------------------------------- pair placement
// Ranks are cut into groups of kGroupRanks. One count kernel (a block per
// group) forms the group's pairs per tile, tc[v][g][t] (scanned over the groups
// into toff: the group's first position in the tile), and per tile row,
// gsum[v][y][g] (whose sums over the groups are the row totals). Placement (a
// block per (group, row)) lays the group's runs in the row out in LDS and puts
// each pair at its tile's cursor, so every tile's run of a group leaves as
// contiguous stores; nothing per pair is staged in global memory.
struct Bins {
    int64_t N;
    int32_t V, G, T, tiles_x, tiles_y, seg_g, nseg_g, xbits;
};
constexpr int kGroupRanks = 4096;             // depth ranks per group
constexpr int kMaxSegs = 32;                  // at most this many segments per column scan

// The group counts' column scan goes by segments of seg_g groups: the count
// kernel adds each segment's sums (segt[v][seg][t]), the tile kernel turns them
// into exclusive prefixes in place, and every group's first position in tile t
// is toff[v][g][t] = tile base + (pairs of the groups before g), the tile base
// being rbase[v][y] + trel[v][t].
__global__ __launch_bounds__(256) void k_tile_offsets(const uint32_t* __restrict__ tc,
                                                      const uint32_t* __restrict__ segt,
                                                      const int64_t* __restrict__ rbase,
                                                      const uint32_t* __restrict__ trel, Bins B,
                                                      uint32_t* __restrict__ toff) {
    const int t = blockIdx.x * 256 + threadIdx.x, seg = blockIdx.y, v = blockIdx.z;
    if (t >= B.T) return;
    const int64_t vt = (int64_t)v * B.T + t;
    uint32_t run = (uint32_t)rbase[(int64_t)v * B.tiles_y + t / B.tiles_x] + trel[vt] +
                   segt[((int64_t)v * B.nseg_g + seg) * B.T + t];
    const int g0 = seg * B.seg_g, g1 = min(B.G, g0 + B.seg_g);
#pragma unroll 8
    for (int g = g0; g < g1; ++g) {
        const int64_t i = ((int64_t)v * B.G + g) * B.T + t;
        toff[i] = run;
        run += tc[i];
    }
}

// Turns the nseg (<= kMaxSegs) segment sums p[0], p[stride], ... into
// exclusive prefixes in place and returns their total. All loads are issued
// before the first store.
__device__ inline uint32_t seg_prefix(uint32_t* __restrict__ p, int64_t stride, int nseg) {
    uint32_t x[kMaxSegs];
#pragma unroll
    for (int k = 0; k < kMaxSegs; ++k) x[k] = k < nseg ? p[k * stride] : 0u;
    uint32_t run = 0;
#pragma unroll
    for (int k = 0; k < kMaxSegs; ++k) {
        if (k < nseg) p[k * stride] = run;
        run += x[k];
    }
    return run;
}

// A block per (view, row): per tile, the segment sums become exclusive prefixes
// in place and give the tile's total; trel = exclusive scan of the row's tile
// totals (the tile's start relative to the row's), rtot = the row's total. The
// block that finishes last (a counter, cleared with the control words) then
// forms the row bases, an exclusive scan of the row totals over (view, row),
// and the number of pairs.
__global__ __launch_bounds__(256) void k_tile_bases(uint32_t* __restrict__ segt, Bins B,
                                                    uint32_t* __restrict__ trel, uint32_t* __restrict__ rtot,
                                                    uint32_t* __restrict__ rows_done,
                                                    int64_t* __restrict__ rbase, int64_t* __restrict__ n_pairs,
                                                    uint32_t* __restrict__ rcov, uint32_t* __restrict__ rltot,
                                                    int64_t* __restrict__ rlbase) {
    __shared__ uint32_t wsum[4];
    __shared__ int64_t wsum64[4];
    __shared__ bool s_last;
    const int y = blockIdx.x, v = blockIdx.y, lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t run = 0;
    const int64_t t0 = (int64_t)v * B.T + (int64_t)y * B.tiles_x;
    for (int x0 = 0; x0 < B.tiles_x; x0 += 256) {
        const int x = x0 + threadIdx.x;
        uint32_t c = 0;
        if (x < B.tiles_x) c = seg_prefix(segt + (int64_t)v * B.nseg_g * B.T + (int64_t)y * B.tiles_x + x, B.T, B.nseg_g);
        const uint32_t inc = wave_incl_scan(c);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = run, all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) pre += wsum[k];
            all += wsum[k];
        }
        if (x < B.tiles_x) trel[t0 + x] = pre + inc - c;
        run += all;
        __syncthreads();
    }
    // the row's list of covering splats: every group's first entry in it (an
    // exclusive scan of the cover counts over the groups, in place) and its length
    uint32_t lrun = 0;
    uint32_t* rc = rcov + ((int64_t)v * B.tiles_y + y) * B.G;
    for (int g0 = 0; g0 < B.G; g0 += 256) {
        const int g = g0 + threadIdx.x;
        const uint32_t c = g < B.G ? rc[g] : 0u;
        const uint32_t inc = wave_incl_scan(c);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = lrun, all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) pre += wsum[k];
            all += wsum[k];
        }
        if (g < B.G) rc[g] = pre + inc - c;
        lrun += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        rtot[(int64_t)v * B.tiles_y + y] = run;
        rltot[(int64_t)v * B.tiles_y + y] = lrun;
        __threadfence();
        s_last = atomicAdd(rows_done, 1u) == gridDim.x * gridDim.y - 1;
    }
    __syncthreads();
    if (!s_last) return;
    __threadfence();   // every block's row total is visible past its counter increment
    const int64_t nr = (int64_t)B.V * B.tiles_y;
    int64_t carry = 0;
    for (int64_t b0 = 0; b0 < nr; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t tot = i < nr ? (int64_t)rtot[i] : 0;
        int64_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        if (lane == 63) wsum64[w] = inc;
        __syncthreads();
        int64_t pre = carry, all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) pre += wsum64[k];
            all += wsum64[k];
        }
        if (i < nr) rbase[i] = pre + inc - tot;
        carry += all;
        __syncthreads();
    }
    if (threadIdx.x == 0) *n_pairs = carry;
    // the same over the row lists' lengths: where each row's list starts
    int64_t lcarry = 0;
    for (int64_t b0 = 0; b0 < nr; b0 += 256) {
        const int64_t i = b0 + threadIdx.x;
        const int64_t tot = i < nr ? (int64_t)rltot[i] : 0;
        int64_t inc = tot;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const int64_t u = __shfl_up(inc, d, 64);
            if (lane >= d) inc += u;
        }
        if (lane == 63) wsum64[w] = inc;
        __syncthreads();
        int64_t pre = lcarry, all = 0;
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            if (k < w) pre += wsum64[k];
            all += wsum64[k];
        }
        if (i < nr) rlbase[i] = pre + inc - tot;
        lcarry += all;
        __syncthreads();
    }
}

// The counts of one group (a block per (group, view)), band by band of tile
// rows, from a difference array in LDS: every splat of the group adds +1 / -1
// at the four corners of its rect; prefix sums down the columns, then along the
// rows, give the group's pairs in every tile: tc[v][g][t], also added into the
// tile's sum over the group's segment of the column scan (segt, cleared
// beforehand), and the group's pairs per row, gsum[v][y][g]. The group's rects
// are gathered in depth order once (and written to srect for the placement).
constexpr int kGcThreads = 1024;
constexpr int kGcItems = kGroupRanks / kGcThreads;
constexpr int kGcBand = 64;                       // rows per band at most (one lane each)
constexpr size_t kGcLds = 48 * 1024;              // LDS budget of the difference array

__global__ __launch_bounds__(kGcThreads) void k_count(const uint32_t* __restrict__ order,
                                                     const uint2* __restrict__ crect, Bins B, int band,
                                                     uint2* __restrict__ srect, uint32_t* __restrict__ gsum,
                                                     uint32_t* __restrict__ tc, uint32_t* __restrict__ segt,
                                                     uint32_t* __restrict__ rcov) {
    extern __shared__ uint32_t d[];   // [band + 1][tiles_x + 1], then [tiles_y + 1] for the row covers
    const int g = blockIdx.x, v = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    constexpr int NW = kGcThreads / 64;
    const int TX = B.tiles_x, W1 = TX + 1;
    const int64_t r0 = (int64_t)g * kGroupRanks;
    const int ns = (int)min((int64_t)kGroupRanks, B.N - r0);
    uint2 rr[kGcItems];
#pragma unroll
    for (int k = 0; k < kGcItems; ++k) {
        const int idx = k * kGcThreads + (int)threadIdx.x;
        rr[k] = make_uint2(0u, 0u);
        if (idx < ns) {
            const int64_t r = (int64_t)v * B.N + r0 + idx;
            rr[k] = crect[(int64_t)v * B.N + order[r]];
            srect[r] = rr[k];
        }
    }
    // how many of the group's splats cover each tile row: +1 at y0, -1 at y1,
    // summed down the rows at the end
    uint32_t* rd = d + (size_t)(band + 1) * W1;
    for (int i = threadIdx.x; i <= B.tiles_y; i += kGcThreads) rd[i] = 0u;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kGcItems; ++k) {
        const int x0 = (int)(rr[k].x & 0xffffu), x1 = (int)(rr[k].x >> 16);
        const int y0 = (int)(rr[k].y & 0xffffu), y1 = (int)(rr[k].y >> 16);
        if (x0 < x1 && y0 < y1) {
            atomicAdd(&rd[y0], 1u);
            atomicSub(&rd[y1], 1u);
        }
    }
    uint32_t* out = tc + ((int64_t)v * B.G + g) * B.T;
    uint32_t* sg = segt + ((int64_t)v * B.nseg_g + g / B.seg_g) * B.T;
    for (int yb0 = 0; yb0 < B.tiles_y; yb0 += band) {
        const int yb1 = min(B.tiles_y, yb0 + band), H = yb1 - yb0;
        for (int i = threadIdx.x; i < (H + 1) * W1; i += kGcThreads) d[i] = 0u;
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kGcItems; ++k) {
            const int x0 = (int)(rr[k].x & 0xffffu), x1 = (int)(rr[k].x >> 16);
            const int y0 = max((int)(rr[k].y & 0xffffu), yb0) - yb0, y1 = min((int)(rr[k].y >> 16), yb1) - yb0;
            if (x0 < x1 && y0 < y1) {
                atomicAdd(&d[y0 * W1 + x0], 1u);
                atomicSub(&d[y0 * W1 + x1], 1u);
                atomicSub(&d[y1 * W1 + x0], 1u);
                atomicAdd(&d[y1 * W1 + x1], 1u);
            }
        }
        __syncthreads();
        // down the columns (a wave per column, a lane per row)
        for (int x = w; x < TX; x += NW) {
            const uint32_t val = lane < H ? d[lane * W1 + x] : 0u;
            const uint32_t inc = wave_incl_scan(val);
            if (lane < H) d[lane * W1 + x] = inc;
        }
        __syncthreads();
        // along the rows (a wave per row, lanes over columns); the row's total
        // is the group's pairs in the row
        for (int y = w; y < H; y += NW) {
            uint32_t carry = 0, rowsum = 0;
            for (int xc = 0; xc < TX; xc += 64) {
                const int x = xc + lane;
                const uint32_t val = x < TX ? d[y * W1 + x] : 0u;
                const uint32_t inc = wave_incl_scan(val);
                const uint32_t c = carry + inc;   // the tile's count
                if (x < TX) {
                    const int64_t t = (int64_t)(yb0 + y) * TX + x;
                    out[t] = c;
                    if (c) atomicAdd(sg + t, c);
                    rowsum += c;
                }
                carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
            }
            rowsum = wave_incl_scan(rowsum);   // lane 63: the row's total
            if (lane == 63) gsum[((int64_t)v * B.tiles_y + yb0 + y) * B.G + g] = rowsum;
        }
        __syncthreads();
    }
    // the row covers: a running sum down the rows (one wave)
    if (w == 0) {
        uint32_t carry = 0;
        for (int y0 = 0; y0 < B.tiles_y; y0 += 64) {
            const int y = y0 + lane;
            const uint32_t inc = wave_incl_scan(y < B.tiles_y ? rd[y] : 0u);
            if (y < B.tiles_y) rcov[((int64_t)v * B.tiles_y + y) * B.G + g] = carry + inc;
            carry += (uint32_t)__builtin_amdgcn_readlane((int)inc, 63);
        }
    }
}

// Row lists, a block per (group, view): for every tile row, the group's
// splats that cover it, in depth-rank order, each as (splat id, its rect's
// columns x0 | x1 << 16), written at the row list's place for the group (the
// bin's cover counts, scanned). Within a band of up to 64 rows, every (row,
// rank slot, wave) gets the 64-bit mask of its covering lanes (each lane marks
// its rows in a word, and a bit transpose over the wave turns the 64 words
// into the 64 rows' masks); a scan of their counts per row gives each wave's
// first place, a popcount below the lane its place.
constexpr int kRwThreads = 1024;
constexpr int kRwItems = kGroupRanks / kRwThreads;   // ranks per thread (rank = slot * 1024 + thread)
constexpr int kRwSlots = kRwItems * (kRwThreads / 64);   // (slot, wave) pairs, in rank order
constexpr int kRwPer = kRwSlots / 64;                      // of them per lane in the per-row scan
constexpr int kRwBand = 4096 / kRwSlots;                  // rows per band (~49 KB of masks and places)
static_assert(kRwSlots % 64 == 0, "the per-row scan gives each lane whole (slot, wave) pairs");

// 64x64 bit-matrix transpose over a wave: lane i's word is row i; on return
// lane j's word holds column j (bit i = bit j of lane i's word). Each stage
// swaps the off-diagonal blocks of one bit of the row and column indices.
__device__ inline uint64_t wave_transpose64(uint64_t r) {
    const int lane = (int)(threadIdx.x & 63u);
    constexpr uint64_t keep[6] = {0x00000000ffffffffull, 0x0000ffff0000ffffull, 0x00ff00ff00ff00ffull,
                                  0x0f0f0f0f0f0f0f0full, 0x3333333333333333ull, 0x5555555555555555ull};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
        const int s = 32 >> k;
        const uint64_t m = keep[k];
        const uint64_t p = __shfl_xor(r, s, 64);
        r = (lane & s) ? ((r & ~m) | ((p >> s) & m)) : ((r & m) | ((p & m) << s));
    }
    return r;
}

__device__ inline uint64_t lanes_below() {
    const int lane = (int)(threadIdx.x & 63u);
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

__global__ __launch_bounds__(kRwThreads) void k_rows(const uint2* __restrict__ srect, const uint32_t* __restrict__ order,
                                                    const uint32_t* __restrict__ rcov,
                                                    const int64_t* __restrict__ rlbase, Bins B,
                                                    const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                    uint2* __restrict__ rows) {
    // rows padded by one word: the lanes of a wave index rows with a common slot,
    // so an unpadded power-of-two row stride would put them all in one LDS bank
    __shared__ uint64_t mask[kRwBand][kRwSlots + 1];
    __shared__ uint32_t wb[kRwBand][kRwSlots + 1];
    __shared__ int64_t rbeg[kRwBand];
    const int g = blockIdx.x, v = blockIdx.y;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t n = *n_pairs;
    if (!(n >= 0 && n <= capacity)) return;   // nothing is placed: the lists are not needed
    const int64_t r0 = (int64_t)g * kGroupRanks;
    const int ns = (int)min((int64_t)kGroupRanks, B.N - r0);
    uint2 rr[kRwItems];
    uint32_t id[kRwItems];
#pragma unroll
    for (int k = 0; k < kRwItems; ++k) {
        const int idx = k * kRwThreads + (int)threadIdx.x;
        rr[k] = make_uint2(0u, 0u);
        id[k] = 0u;
        if (idx < ns) {
            const int64_t r = (int64_t)v * B.N + r0 + idx;
            rr[k] = srect[r];
            id[k] = order[r];
        }
    }
    const uint64_t below = lanes_below();
    for (int yb0 = 0; yb0 < B.tiles_y; yb0 += kRwBand) {
        const int nb = min(kRwBand, B.tiles_y - yb0);
        // every lane marks the band's rows it covers in one 64-bit word; the
        // wave's words, transposed, give every row the mask of its covering lanes
#pragma unroll
        for (int k = 0; k < kRwItems; ++k) {
            const int x0 = (int)(rr[k].x & 0xffffu), x1 = (int)(rr[k].x >> 16);
            const int y0 = max((int)(rr[k].y & 0xffffu), yb0) - yb0, y1 = min((int)(rr[k].y >> 16), yb0 + nb) - yb0;
            // rows [y0, y1) of the band, 0 <= y0 and y1 <= nb <= 64 (none when y0 >= y1)
            const bool any = x0 < x1 && y0 < y1;
            const uint64_t hi = y1 >= 64 ? ~0ull : (1ull << (any ? y1 : 0)) - 1ull;
            const uint64_t lo = (1ull << (any ? y0 : 0)) - 1ull;
            const uint64_t rowbits = any ? (hi & ~lo) : 0ull;
            const uint64_t cov = wave_transpose64(rowbits);
            if (lane < nb) mask[lane][k * (kRwThreads / 64) + w] = cov;
        }
        if ((int)threadIdx.x < nb) {
            const int64_t vy = (int64_t)v * B.tiles_y + yb0 + threadIdx.x;
            rbeg[threadIdx.x] = rlbase[vy] + rcov[vy * B.G + g];
        }
        __syncthreads();
        for (int yy = w; yy < nb; yy += kRwThreads / 64) {
            uint32_t c[kRwPer], t = 0;
#pragma unroll
            for (int q = 0; q < kRwPer; ++q) {
                c[q] = (uint32_t)__popcll(mask[yy][kRwPer * lane + q]);
                t += c[q];
            }
            uint32_t pre = wave_incl_scan(t) - t;
#pragma unroll
            for (int q = 0; q < kRwPer; ++q) {
                wb[yy][kRwPer * lane + q] = pre;
                pre += c[q];
            }
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kRwItems; ++k) {
            const int x0 = (int)(rr[k].x & 0xffffu), x1 = (int)(rr[k].x >> 16);
            const int y0 = max((int)(rr[k].y & 0xffffu), yb0), y1 = min((int)(rr[k].y >> 16), yb0 + nb);
            if (x0 >= x1) continue;
            for (int y = y0; y < y1; ++y) {
                const int yy = y - yb0, sl = k * (kRwThreads / 64) + w;
                const int64_t pos = rbeg[yy] + wb[yy][sl] + __popcll(mask[yy][sl] & below);
                rows[pos] = make_uint2(id[k], rr[k].x);
            }
        }
        __syncthreads();
    }
}

// Pair placement, a block per (view, tile row, group): the group's row list (its
// splats covering the row, in rank order) goes out as pairs, each splat to
// every tile x0..x1-1 of its run, at the tile's cursor (the group's first
// position in the tile, from the bin's counts). The list goes by chunks of 128
// entries. A chunk's pairs, numbered entry by entry (a block scan of the run
// widths), are cut into equal consecutive shares, one per thread, so that wide
// and narrow runs cost every thread alike (the entry whose run holds a share's
// first pair marks itself as the share's first); each thread walks its share twice.
// The first walk sets, per pair, the entry's bit in the 64-bit mask of (the
// entry's wave, the pair's column) (LDS atomic ORs). A column pass turns the
// masks into each (wave, column)'s first place and advances the cursors. The
// second walk puts each entry's splat id at its place in each of its columns:
// the first place of its (wave, column) plus its wave's entries below it in
// the mask. Entries are in rank order within a mask, masks within the chunk
// and chunks within the list, so every tile's run of the group stays in rank
// order. Blocks of group 0 also write the row's tile ranges, [0, 0) when empty
// and all empty when the pairs exceed the capacity.
constexpr int kPcThreads = 128;
constexpr int kPcWaves = kPcThreads / 64;
constexpr int kPcStage = 1024;   // pairs of a chunk staged for the coalesced write-out

// The next entry after i with a nonempty run (one exists when a pair is left).
__device__ inline int next_run(const uint32_t* ecol, int i, uint32_t& x, uint32_t& xe) {
    uint32_t c;
    do {
        c = ecol[++i];
    } while ((c >> 16) <= (c & 0xffffu));
    x = c & 0xffffu;
    xe = c >> 16;
    return i;
}

__global__ __launch_bounds__(kPcThreads) void k_place(const uint2* __restrict__ rows,
                                                     const uint32_t* __restrict__ rcov,
                                                     const uint32_t* __restrict__ rltot,
                                                     const int64_t* __restrict__ rlbase,
                                                     const uint32_t* __restrict__ off,
                                                     const int64_t* __restrict__ rbase,
                                                     const uint32_t* __restrict__ trel,
                                                     const uint32_t* __restrict__ rtot, Bins B,
                                                     const int64_t* __restrict__ n_pairs, int64_t capacity,
                                                     uint32_t* __restrict__ ids, int32_t* __restrict__ ranges) {
    extern __shared__ __align__(16) uint64_t lds64[];
    const int TX = B.tiles_x;
    uint64_t* mask = lds64;                                              // [kPcWaves][TX]
    uint32_t* cur = reinterpret_cast<uint32_t*>(mask + kPcWaves * TX);   // [TX]
    uint32_t* wbase = cur + TX;                                          // [kPcWaves][TX]
    uint32_t* eid = wbase + kPcWaves * TX;                               // [kPcThreads] the chunk's splat ids
    uint32_t* ecol = eid + kPcThreads;                                   // [kPcThreads] their runs x0 | x1 << 16
    uint32_t* pst = ecol + kPcThreads;                                   // [kPcThreads] their first pairs
    uint32_t* fe = pst + kPcThreads;                                     // [kPcThreads] each share's first entry
    uint32_t* wsum = fe + kPcThreads;                                    // [2][kPcWaves]
    uint32_t* cst = wsum + 2 * kPcWaves;                                 // [TX] place - staging slot per column
    uint32_t* sid = cst + TX;                                            // [kPcStage] staged splat ids
    uint16_t* scol = reinterpret_cast<uint16_t*>(sid + kPcStage);       // [kPcStage] and their columns
    // workgroups go to the 8 XCDs round-robin by linear id: block b runs on XCD
    // b % 8, and XCD x takes the tile rows x, x + 8, ... with all their groups in
    // rank order, so every tile's list (the runs of all the groups, one after
    // another) is written through one XCD's L2
    const int xcd = (int)(blockIdx.x & 7u), m = (int)(blockIdx.x >> 3), v = blockIdx.y;
    const int j = m / B.G, g = m - j * B.G, y = xcd + 8 * j;
    if (y >= B.tiles_y) return;
    const int t = (int)threadIdx.x, lane = t & 63, w = t >> 6;
    const int64_t n = *n_pairs;
    const bool fits = n >= 0 && n <= capacity;
    const int64_t vy = (int64_t)v * B.tiles_y + y;
    if (g == 0) {
        const int64_t rb = rbase[vy];
        for (int x = t; x < TX; x += kPcThreads) {
            const int64_t i = (int64_t)v * B.T + (int64_t)y * TX + x;
            const int64_t b = rb + trel[i], e = rb + (x + 1 < TX ? trel[i + 1] : rtot[vy]);
            const bool any = fits && e > b;
            ranges[2 * i] = any ? (int32_t)b : 0;
            ranges[2 * i + 1] = any ? (int32_t)e : 0;
        }
    }
    if (!fits) return;
    const int64_t lb = rlbase[vy];
    const int64_t beg = lb + rcov[vy * B.G + g];
    const int64_t end = lb + (g + 1 < B.G ? rcov[vy * B.G + g + 1] : rltot[vy]);
    if (end <= beg) return;
    const int cnt = (int)(end - beg);
    const uint32_t* orow = off + ((int64_t)v * B.G + g) * B.T + (int64_t)y * TX;
    for (int x = t; x < TX; x += kPcThreads) cur[x] = orow[x];
    uint2 en = t < cnt ? rows[beg + t] : make_uint2(0u, 0u);   // this thread's entry of the first chunk
    for (int c0 = 0; c0 < cnt; c0 += kPcThreads) {
        // (each thread's cursors are its own; the barrier before the last chunk's
        // copy-out ended every other use of the arrays written from here on)
        for (int i = t; i < kPcWaves * TX; i += kPcThreads) mask[i] = 0ull;
        const uint2 e = en;
        // the next chunk's entry, in flight while this chunk is placed
        if (c0 + kPcThreads < cnt) en = c0 + kPcThreads + t < cnt ? rows[beg + c0 + kPcThreads + t] : make_uint2(0u, 0u);
        const uint32_t ex0 = e.y & 0xffffu, ex1 = e.y >> 16;
        const uint32_t wd = ex1 > ex0 ? ex1 - ex0 : 0u;
        eid[t] = e.x;
        ecol[t] = e.y;
        const uint32_t inc = wave_incl_scan(wd);
        if (lane == 63) wsum[w] = inc;
        __syncthreads();
        uint32_t pre = 0, np = 0;
#pragma unroll
        for (int k = 0; k < kPcWaves; ++k) {
            if (k < w) pre += wsum[k];
            np += wsum[k];
        }
        const uint32_t p0 = pre + inc - wd;
        pst[t] = p0;
        // thread s's share is pairs [s * share, (s + 1) * share) of the chunk's np;
        // the entry whose run holds a share's first pair marks itself as its first
        const uint32_t share = (np + kPcThreads - 1) / kPcThreads;
        if (wd > 0)
            for (uint32_t sh = (p0 + share - 1) / share; sh * share < p0 + wd; ++sh) fe[sh] = (uint32_t)t;
        __syncthreads();
        // this thread's share [q0, q1); its first pair's entry and column
        const uint32_t q0 = min(np, (uint32_t)t * share), q1 = min(np, q0 + share);
        int i0 = 0;
        uint32_t x0 = 0, xe0 = 0;
        if (q0 < q1) {
            i0 = (int)fe[t];
            const uint32_t c = ecol[i0];
            x0 = (c & 0xffffu) + (q0 - pst[i0]);
            xe0 = c >> 16;
        }
        {
            int i = i0;
            uint32_t x = x0, xe = xe0;
            for (uint32_t q = q0; q < q1; ++q) {
                atomicOr((unsigned long long*)&mask[(i >> 6) * TX + (int)x], (unsigned long long)(1ull << (i & 63)));
                if (++x == xe && q + 1 < q1) i = next_run(ecol, i, x, xe);
            }
        }
        __syncthreads();
        // the chunk's ids go out in place order: staged in LDS by (column, place)
        // with their columns, then copied to consecutive addresses per column; a
        // chunk of more pairs than the staging holds writes every id at its place
        // directly. Per column: each wave's first place, the cursor advanced past
        // the chunk, and the column's first slot in the staging order; staged,
        // each (wave, column) base is kept as its first staging slot and the
        // column's first slot as the difference place - slot of its pairs, so that
        // a pair needs one LDS round trip and a copy one more
        const bool staged = np <= (uint32_t)kPcStage;
        uint32_t carry = 0;
        for (int x0c = 0, par = 0; x0c < TX; x0c += kPcThreads, par ^= kPcWaves) {
            const int x = x0c + t;
            uint32_t c0 = 0, c = 0, cw[kPcWaves];
            if (x < TX) {
                c0 = c = cur[x];
#pragma unroll
                for (int ww = 0; ww < kPcWaves; ++ww) {
                    cw[ww] = c;
                    c += (uint32_t)__popcll(mask[ww * TX + x]);
                }
                cur[x] = c;
            }
            const uint32_t cn = c - c0;
            const uint32_t inc = wave_incl_scan(cn);
            // the passes alternate between two halves of wsum, so one barrier
            // separates a pass's reads from the next writes of the same half
            if (lane == 63) wsum[par + w] = inc;
            __syncthreads();
            uint32_t pre = carry, all = 0;
#pragma unroll
            for (int k = 0; k < kPcWaves; ++k) {
                if (k < w) pre += wsum[par + k];
                all += wsum[par + k];
            }
            if (x < TX) {
                const uint32_t s0 = pre + inc - cn;
#pragma unroll
                for (int ww = 0; ww < kPcWaves; ++ww) wbase[ww * TX + x] = staged ? s0 + (cw[ww] - c0) : cw[ww];
                cst[x] = c0 - s0;
            }
            carry += all;
        }
        __syncthreads();
        {
            int i = i0;
            uint32_t x = x0, xe = xe0;
            for (uint32_t q = q0; q < q1; ++q) {
                const int s = (i >> 6) * TX + (int)x;
                const uint64_t below = (1ull << (i & 63)) - 1ull;
                const uint32_t at = wbase[s] + (uint32_t)__popcll(mask[s] & below);   // staging slot, or place
                if (staged) {
                    sid[at] = eid[i];
                    scol[at] = (uint16_t)x;
                } else {
                    ids[at] = eid[i];
                }
                if (++x == xe && q + 1 < q1) i = next_run(ecol, i, x, xe);
            }
        }
        __syncthreads();
        if (staged) {
            // four copies in flight per thread
            for (uint32_t o0 = (uint32_t)t; o0 < np; o0 += 4 * kPcThreads) {
                uint32_t xs[4], vs[4];
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t o = o0 + u * kPcThreads;
                    xs[u] = o < np ? scol[o] : 0u;
                    vs[u] = o < np ? sid[o] : 0u;
                }
#pragma unroll
                for (int u = 0; u < 4; ++u) {
                    const uint32_t o = o0 + u * kPcThreads;
                    const uint32_t d = cst[xs[u]];
                    if (o < np) ids[o + d] = vs[u];
                }
            }
        }
    }
}

// ---------------------------------------------------------------- host side
// Region at the front of the workspace, cleared at the start of every bin:
// counter words (the last one counts finished tile rows), digit totals and the
// key range.
struct Ctl {
    uint32_t* ticket;
    uint32_t* ghist;
    uint32_t* krange;   // per view: largest key, largest complemented key
    uint32_t* offs;   // per (view, digit, block) counts, then places (not cleared: written before read)
    int64_t clear_words;
};

Bins bins_of(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y) {
    Bins B;
    B.N = N;
    B.V = V;
    B.G = (int32_t)ceil_div(N, kGroupRanks);
    B.tiles_x = tiles_x;
    B.tiles_y = tiles_y;
    B.T = tiles_x * tiles_y;
    B.seg_g = (int32_t)std::max<int64_t>(16, ceil_div(B.G, kMaxSegs));
    B.nseg_g = (int32_t)std::max<int64_t>(1, ceil_div(B.G, B.seg_g));
    int bits = 1;
    while ((1 << bits) < tiles_x) ++bits;
    B.xbits = bits;
    return B;
}

struct BinWs {
    Ctl ctl;
    uint32_t *ka, *kb, *va, *vb;
    uint2 *crect, *srect;   // rects by splat id, and in depth order
    uint2* kpart;           // per (view, wave of 64 splats) key-range partials of a fused projection
    uint32_t *gsum, *rtot;
    int64_t* rbase;
    uint32_t *tc, *toff, *segt, *trel;
    uint32_t *rcov, *rltot;   // per (view, row, group): covering splats (then first list entry); per row: list length
    int64_t* rlbase;          // per (view, row): the row list's start
    size_t bytes;
};

BinWs bin_layout(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y, char* base) {
    const int64_t VN = N * V;
    const int64_t bps = ceil_div(N > 0 ? N : 1, kTile);
    const Bins B = bins_of(N, V, tiles_x, tiles_y);
    BinWs w;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b > 0 ? b : 1); return p; };
    // counter words (the tile-row counter of k_tile_bases among them)
    w.ctl.ticket = (uint32_t*)take(4 * (kMaxPasses + 2));
    w.ctl.ghist = (uint32_t*)take(4 * (size_t)V * kMaxPasses * 256);
    w.ctl.krange = (uint32_t*)take(4 * 2 * (size_t)V);
    const size_t ty = (size_t)tiles_y, T = (size_t)B.T;
    // cleared with the control words: the sums the group counts add into
    w.segt = (uint32_t*)take(4 * (size_t)V * B.nseg_g * T);
    w.ctl.clear_words = (int64_t)(o / 8);
    w.ctl.offs = (uint32_t*)take(4 * (size_t)V * bps * 256);
    w.kpart = (uint2*)take(8 * (size_t)V * (size_t)ceil_div(N > 0 ? N : 1, 64));
    w.ka = (uint32_t*)take(4 * VN);
    w.kb = (uint32_t*)take(4 * VN);
    w.va = (uint32_t*)take(4 * VN);
    w.vb = (uint32_t*)take(4 * VN);
    w.crect = (uint2*)take(8 * VN);
    w.srect = (uint2*)take(8 * VN);
    w.gsum = (uint32_t*)take(4 * (size_t)V * ty * B.G);
    w.rtot = (uint32_t*)take(4 * (size_t)V * ty);
    w.rbase = (int64_t*)take(8 * (size_t)V * ty);
    w.tc = (uint32_t*)take(4 * (size_t)V * B.G * T);
    w.toff = (uint32_t*)take(4 * (size_t)V * B.G * T);
    w.trel = (uint32_t*)take(4 * (size_t)V * T);
    w.rcov = (uint32_t*)take(4 * (size_t)V * ty * B.G);
    w.rltot = (uint32_t*)take(4 * (size_t)V * ty);
    w.rlbase = (int64_t*)take(8 * (size_t)V * ty);
    w.bytes = o;
    return w;
}


potr_status radix_pass(const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, uint32_t* vfinal,
                       const Seg& g, int segs, const Pass& P, const uint32_t* krange, hipStream_t s) {
    const dim3 grid((unsigned)g.bps, (unsigned)segs);
    hipLaunchKernelGGL(k_pass_count, grid, dim3(256), 0, s, kin, g, P, krange);
    hipLaunchKernelGGL(k_pass_scan, dim3(256, (unsigned)segs), dim3(256), 0, s, g, P, krange);
    hipLaunchKernelGGL(k_pass_scatter, grid, dim3(kSwThreads), 0, s, kin, kout, vin, vout, vfinal, g, P, krange);
    return check_launch("k_pass_count / k_pass_scan / k_pass_scatter");
}

// rows per band of the group counts' difference array, and its LDS bytes
int gc_band(int tiles_x) {
    const int rows = (int)(kGcLds / (4 * (size_t)(tiles_x + 1))) - 1;
    return std::max(1, std::min(kGcBand, rows));
}
size_t gc_lds(int band, int tiles_x, int tiles_y) {
    return (size_t)(band + 1) * (tiles_x + 1) * 4 + (size_t)(tiles_y + 1) * 4;
}

// LDS of the placement: per wave and tile column a 64-bit mask and a first
// place, a cursor and a first staging slot per column, per chunk entry its id,
// run and first pair, per thread its share's first entry, and the staged ids
// and their columns (11.1 KB at 100 columns, 72.0 KB at 2048)
size_t place_lds(const Bins& B) {
    return (size_t)B.tiles_x * (kPcWaves * 8 + kPcWaves * 4 + 4 + 4) + 4 * kPcThreads * 4 + 2 * kPcWaves * 4 +
           (size_t)kPcStage * 6;
}


}  // namespace

size_t bin_workspace_bytes(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y) {
    return bin_layout(N, V, tiles_x, tiles_y, nullptr).bytes;
}

// The row lists: one 8-byte entry per (splat, covered tile row), at most one
// per pair, so `capacity` entries always suffice.
size_t sort_workspace_bytes(int64_t capacity) { return align_up((size_t)(capacity > 0 ? capacity : 1) * 8); }

BinKeys bin_keys(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg, void* ws) {
    const BinWs w = bin_layout(N, V, tiles_x(cam0, cfg), tiles_y(cam0, cfg), (char*)ws);
    return BinKeys{w.ka, w.crect, w.kpart, ceil_div(N > 0 ? N : 1, 64)};
}

potr_status launch_bin(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                       const potr_proj* proj, void* ws, uint32_t* order, int64_t* n_pairs, hipStream_t s,
                       bool keys_ready) {
    const int txs = tiles_x(cam0, cfg), tys = tiles_y(cam0, cfg);
    BinWs w = bin_layout(N, V, txs, tys, (char*)ws);
    const Bins B = bins_of(N, V, txs, tys);
    const unsigned cb = (unsigned)std::min<int64_t>(ceil_div(w.ctl.clear_words, 256), 4096);
    hipLaunchKernelGGL(k_clear, dim3(cb), dim3(256), 0, s, (uint64_t*)w.ctl.ticket, w.ctl.clear_words);
    potr_status st = check_launch("k_clear");
    if (st != POTR_OK) return st;
    if (N > 0) {
        // stable per-view sort of the 32-bit depth keys by key - min: as many
        // 8-bit passes as the view's span of keys needs (the rest return at once)
        Seg g{N, nullptr, 0, (int32_t)ceil_div(N, kTile)};
        const dim3 kg((unsigned)ceil_div(N, kHistThreads * kHistItems), V);
        if (keys_ready) {
            // keys and rects written by the projection: only the key range is left
            const int64_t pv = ceil_div(N, 64);
            const dim3 kr((unsigned)std::min<int64_t>(64, ceil_div(pv, kHistThreads)), V);
            hipLaunchKernelGGL(k_krange, kr, dim3(kHistThreads), 0, s, (const uint2*)w.kpart, pv, w.ctl.krange);
            st = check_launch("k_krange");
        } else {
            hipLaunchKernelGGL(k_keys, kg, dim3(kHistThreads), 0, s, proj, N, w.ka, w.crect, w.ctl.krange);
            st = check_launch("k_keys");
        }
        if (st != POTR_OK) return st;
        uint32_t *kin = w.ka, *kout = w.kb;
        const uint32_t* vin = nullptr;
        uint32_t* vbuf[2] = {w.va, w.vb};   // never the output: a view's last pass may be any of them
        for (int pass = 0; pass < kMaxPasses; ++pass) {
            Pass P{pass, 8 * pass, 8, w.ctl.ghist + pass * 256, w.ctl.offs};
            st = radix_pass(kin, kout, vin, vbuf[pass & 1], order, g, V, P, w.ctl.krange, s);
            if (st != POTR_OK) return st;
            vin = vbuf[pass & 1];
            uint32_t* t = kin;
            kin = kout;
            kout = t;
        }
        const int band = gc_band(txs);
        hipLaunchKernelGGL(k_count, dim3(B.G, V), dim3(kGcThreads), gc_lds(band, txs, tys), s, (const uint32_t*)order,
                           (const uint2*)w.crect, B, band, w.srect, w.gsum, w.tc, w.segt, w.rcov);
        st = check_launch("k_count");
        if (st != POTR_OK) return st;
    }
    // tile starts within their rows and row totals, then row bases over
    // (view, row), the pair count, and every group's first position per tile
    hipLaunchKernelGGL(k_tile_bases, dim3(tys, V), dim3(256), 0, s, w.segt, B, w.trel, w.rtot, w.ctl.ticket + kMaxPasses,
                       w.rbase, n_pairs, w.rcov, w.rltot, w.rlbase);
    st = check_launch("k_tile_bases");
    if (st != POTR_OK || N == 0) return st;
    hipLaunchKernelGGL(k_tile_offsets, dim3((unsigned)ceil_div(B.T, 256), B.nseg_g, V), dim3(256), 0, s,
                       (const uint32_t*)w.tc, (const uint32_t*)w.segt, (const int64_t*)w.rbase,
                       (const uint32_t*)w.trel, B, w.toff);
    return check_launch("k_tile_offsets");
}

potr_status launch_sort(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                        const potr_proj* proj, const uint32_t* order, void* ws, const int64_t* n_pairs,
                        int64_t capacity, void* sort_ws, uint32_t* sorted_ids, int32_t* tile_ranges,
                        hipStream_t s) {
    const int txs = tiles_x(cam0, cfg), tys = tiles_y(cam0, cfg);
    BinWs w = bin_layout(N, V, txs, tys, (char*)ws);
    const Bins B = bins_of(N, V, txs, tys);
    if (N == 0) {
        // no pairs: every tile range is [0, 0)
        const int64_t words = (int64_t)V * B.T;
        hipLaunchKernelGGL(k_clear, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(words, 256), 4096))),
                           dim3(256), 0, s, (uint64_t*)tile_ranges, words);
        return check_launch("k_clear");
    }
    // the row lists, then every (group, row) list to its tiles (and the tile ranges)
    uint2* rows = (uint2*)sort_ws;
    hipLaunchKernelGGL(k_rows, dim3(B.G, V), dim3(kRwThreads), 0, s, (const uint2*)w.srect, order,
                       (const uint32_t*)w.rcov, (const int64_t*)w.rlbase, B, n_pairs, capacity, rows);
    potr_status st = check_launch("k_rows");
    if (st != POTR_OK) return st;
    const dim3 gp((unsigned)(8 * ceil_div(tys, 8) * B.G), V);   // see the XCD mapping in k_place
    hipLaunchKernelGGL(k_place, gp, dim3(kPcThreads), place_lds(B), s, (const uint2*)rows, (const uint32_t*)w.rcov,
                       (const uint32_t*)w.rltot, (const int64_t*)w.rlbase, (const uint32_t*)w.toff,
                       (const int64_t*)w.rbase, (const uint32_t*)w.trel, (const uint32_t*)w.rtot, B, n_pairs,
                       capacity, sorted_ids, tile_ranges);
    return check_launch("k_place");
}

}  // namespace potr
