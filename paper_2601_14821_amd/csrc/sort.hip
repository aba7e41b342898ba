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
// Depth radix passes are one kernel each: a block of 1024 threads x 4 items
// ranks its keys per digit with 64-lane ballots (stable order: wave, item,
// lane), publishes its digit counts, and finds the counts of all blocks before
// it by decoupled look-back over their published words. The passes sort by
// key - min over the view's keys: a view whose keys span fewer than 2^24 (2^16,
// 2^8) values needs three (two, one) passes, and the rest return at once. The
// key range, then the digit totals of the passes needed, come from two reads
// up front. Blocks take their place in
// the chain from an atomic ticket, so a block only ever waits on blocks that
// are already running. Each block sorts its keys in LDS and writes every
// digit's run to consecutive addresses. Every wait is bounded: after
// kSpinLimit polls the block records a fault and goes on (the bin then reports
// n_pairs = -1), so no input can leave a kernel spinning.
#include <algorithm>

#include "common.h"
#include "dpp.h"

namespace potr {
namespace {

constexpr int kThreads = 256;
constexpr int kWaves = kThreads / 64;
constexpr int kSwThreads = 1024;              // depth radix pass: 16 waves x 4 keys per lane
constexpr int kSwItems = 4;
constexpr int kSwWaves = kSwThreads / 64;
constexpr int kTile = kSwThreads * kSwItems;  // keys per block
constexpr int kMaxPasses = 4;
constexpr uint32_t kSpinLimit = 1u << 20;

// ---------------------------------------------------------------- look-back words
// [63:60] pass tag, [59:58] state (1: block aggregate, 2: inclusive prefix), [57:0] count.
// Status arrays are cleared once per call; the tag tells this pass's words from
// those the previous pass left in the same array.
constexpr uint64_t kStAgg = 1, kStInc = 2;
constexpr uint64_t kValMask = (1ull << 58) - 1;

__device__ inline uint64_t st_word(uint32_t tag, uint64_t state, uint64_t v) {
    return ((uint64_t)tag << 60) | (state << 58) | v;
}
__device__ inline void st_put(uint64_t* p, uint64_t w) {
    __hip_atomic_store(p, w, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint64_t st_get(uint64_t* p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ inline uint32_t st_state(uint64_t w, uint32_t tag) {
    return (uint32_t)(w >> 60) == tag ? (uint32_t)((w >> 58) & 3u) : 0u;
}

// Exclusive prefix of one counter over blocks 0..b-1 (words at st[p * stride]):
// adds aggregates walking back until an inclusive prefix is found, reading W
// predecessors per round (their loads are independent, so a round costs one
// memory latency). Aggregates before a not yet published word are taken
// before waiting on it.
template <int W>
__device__ uint64_t look_back(uint64_t* st, int64_t b, int stride, uint32_t tag, uint32_t* fault) {
    uint64_t excl = 0;
    uint32_t spins = 0;
    int64_t hi = b - 1;
    while (hi >= 0) {
        uint64_t wv[W];
#pragma unroll
        for (int k = 0; k < W; ++k) wv[k] = hi - k >= 0 ? st_get(st + (hi - k) * stride) : 0ull;
        int k = 0;
        bool found = false, gap = false;
        for (; k < W; ++k) {
            if (hi - k < 0) {          // before block 0: an inclusive zero
                found = true;
                break;
            }
            const uint32_t s = st_state(wv[k], tag);
            if (s == 0) {
                gap = true;
                break;
            }
            excl += wv[k] & kValMask;
            if (s == kStInc) {
                found = true;
                break;
            }
        }
        if (found) break;
        if (gap) {
            hi -= k;
            if (++spins > kSpinLimit) {
                atomicOr(fault, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        hi -= W;
    }
    return excl;
}

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
    uint32_t tag;             // 1 + pass index
    const uint32_t* ghist;    // this pass's digit totals at ghist[seg * kMaxPasses * 256 + digit]
    uint64_t* status;         // [seg][bps][1 << bits]
    uint32_t* ticket;
    uint32_t* fault;
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

// Radix passes needed for the offsets key - min of one view: 8 bits each, at
// least one (which then also writes the identity order of equal keys).
__device__ inline int passes_of(const uint32_t* krange, int v, uint32_t& kmin) {
    const uint32_t hi = krange[2 * v];
    kmin = ~krange[2 * v + 1];
    const uint32_t span = hi >= kmin ? hi - kmin : 0u;
    const int bits = span ? 32 - __clz((int)span) : 0;
    return max(1, (bits + 7) / 8);
}

// Digit totals of the passes a view needs, over the offsets key - min.
__global__ __launch_bounds__(kHistThreads) void k_digits(const uint32_t* __restrict__ keys, int64_t N,
                                                        const uint32_t* __restrict__ krange,
                                                        uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kMaxPasses][256];
    for (int t = threadIdx.x; t < kMaxPasses * 256; t += kHistThreads) (&h[0][0])[t] = 0;
    __syncthreads();
    const int v = blockIdx.y;
    uint32_t kmin;
    const int np = passes_of(krange, v, kmin);
    const int64_t base = (int64_t)v * N;
    const int64_t e0 = (int64_t)blockIdx.x * (kHistThreads * kHistItems) + threadIdx.x;
    uint32_t d[kHistItems];
#pragma unroll
    for (int k = 0; k < kHistItems; ++k) d[k] = keys[base + min(e0 + (int64_t)k * kHistThreads, N - 1)] - kmin;
#pragma unroll
    for (int k = 0; k < kHistItems; ++k)
        if (e0 + (int64_t)k * kHistThreads < N)
            for (int p = 0; p < np; ++p) atomicAdd(&h[p][(d[k] >> (8 * p)) & 255u], 1u);
    __syncthreads();
    for (int t = threadIdx.x; t < np * 256; t += kHistThreads) {
        const uint32_t c = (&h[0][0])[t];
        if (c) atomicAdd(ghist + (int64_t)v * kMaxPasses * 256 + t, c);
    }
}

// One stable radix pass over the depth keys of every view, by the digits of
// key - min (the view's passes_of decides how many passes it needs; the later
// ones return at once). Values come from vin, or are the element's index when
// vin == nullptr. A view's last pass writes only the values, to vfinal; the
// others write keys to kout and values to vout.
__global__ __launch_bounds__(kSwThreads) void k_sweep(const uint32_t* __restrict__ kin, uint32_t* __restrict__ kout,
                                                    const uint32_t* __restrict__ vin, uint32_t* __restrict__ vout,
                                                    uint32_t* __restrict__ vfinal, Seg g, Pass P,
                                                    const uint32_t* __restrict__ krange) {
    __shared__ uint32_t wcnt[kSwWaves][256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t boff[256];
    __shared__ uint32_t wsum[kSwWaves];
    __shared__ uint32_t s_ticket;
    __shared__ uint32_t s_key[kTile];
    __shared__ uint32_t s_val[kTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t radix = 1u << P.bits, mask = radix - 1;
    if (threadIdx.x == 0) s_ticket = atomicAdd(P.ticket, 1u);
    for (int t = threadIdx.x; t < kSwWaves * 256; t += kSwThreads) (&wcnt[0][0])[t] = 0;
    __syncthreads();
    const int seg = (int)(s_ticket / (uint32_t)g.bps);
    const int64_t b = (int64_t)(s_ticket - (uint32_t)seg * (uint32_t)g.bps);
    uint32_t kmin;
    const int np = passes_of(krange, seg, kmin);
    if (P.pass >= np) return;   // every block of this view returns: nobody waits on them
    const bool last = P.pass == np - 1;
    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.len;
    const int64_t blk0 = b * kTile;
    const int64_t wbase = blk0 + (int64_t)w * (64 * kSwItems);

    // this segment's digit bases: exclusive scan of the pass's digit totals
    const uint32_t gh = threadIdx.x < radix ? P.ghist[(int64_t)seg * kMaxPasses * 256 + threadIdx.x] : 0u;
    const uint32_t dbase = block_excl_scan<kSwThreads>(gh, wsum);

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
        // publish this block's count, then find the counts before it
        uint64_t* st = P.status + ((int64_t)seg * g.bps) * radix + d;
        uint64_t excl = 0;
        if (b == 0) {
            st_put(st, st_word(P.tag, kStInc, run));
        } else {
            st_put(st + b * radix, st_word(P.tag, kStAgg, run));
            excl = look_back<4>(st, b, (int)radix, P.tag, P.fault);
            st_put(st + b * radix, st_word(P.tag, kStInc, excl + run));
        }
        goff[d] = dbase + (uint32_t)excl;
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

// Clears 64-bit words (look-back status, digit totals, key range, tickets).
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
constexpr int kColItems = 8;                  // placement: pairs per thread (2048 per block pass)
// A pair in LDS is one word: tile x << kRankBits | rank of the splat within its group.
constexpr int kRankBits = 12;
static_assert(kGroupRanks == 1 << kRankBits, "a group's ranks fill the rank field");

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
// and the number of pairs (-1 if a depth pass gave up a wait).
__global__ __launch_bounds__(256) void k_tile_bases(uint32_t* __restrict__ segt, Bins B,
                                                    uint32_t* __restrict__ trel, uint32_t* __restrict__ rtot,
                                                    uint32_t* __restrict__ rows_done,
                                                    const uint32_t* __restrict__ fault,
                                                    int64_t* __restrict__ rbase, int64_t* __restrict__ n_pairs) {
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
    if (threadIdx.x == 0) {
        rtot[(int64_t)v * B.tiles_y + y] = run;
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
    if (threadIdx.x == 0) *n_pairs = *fault ? (int64_t)-1 : carry;
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
                                                     uint32_t* __restrict__ tc, uint32_t* __restrict__ segt) {
    extern __shared__ uint32_t d[];   // [band + 1][tiles_x + 1]
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
}

// Pair placement, a block per (view, group, row). The group's splats that cover
// the row, in rank order, each make a run of pairs over the tiles x0..x1-1 of
// their rect; laid back to back these runs are the group's pairs of the row in
// (rank, x) order. Per round of 2048 ranks the covering ranks' runs go to LDS
// as a compact list (a scan of the run widths gives their starts, ballots of
// the cover flags their places in the list);
// per pass of up to 2048 pairs every thread fills eight consecutive slots of
// the pass buffer (one binary search for the run holding its first pair, then a
// walk over the runs; two 16-byte LDS stores) with words (tile x, rank within
// the group), the block ranks them
// stably by tile x (ballots over the x bits, per-wave counters), maps each rank
// to its splat id, sorts in LDS and stores each tile's run at the tile's cursor
// (the group's first position in the tile, advanced per pass).
// Blocks of group 0 also write the row's tile ranges, [0, 0) when empty and all
// empty when the pairs exceed the capacity.
constexpr int kPlRound = 2048;                       // ranks per round
constexpr int kPlSlots = kPlRound / kThreads;        // ranks per lane per round
constexpr int kPlPer = kThreads * kColItems / kThreads;   // pairs each thread expands per pass
static_assert(kPlPer == 8, "the expansion stores a thread's slots as two 16-byte words");

template <int XBITS>
__global__ __launch_bounds__(256) void k_place(const uint2* __restrict__ srect, const uint32_t* __restrict__ gsum,
                                               const uint32_t* __restrict__ off, const int64_t* __restrict__ rbase,
                                               const uint32_t* __restrict__ trel, const uint32_t* __restrict__ rtot,
                                               Bins B, const int64_t* __restrict__ n_pairs, int64_t capacity,
                                               const uint32_t* __restrict__ order, uint32_t* __restrict__ ids,
                                               int32_t* __restrict__ ranges) {
    extern __shared__ __align__(16) uint32_t lds[];
    const int TX = B.tiles_x;
    uint32_t* s_id = lds;                              // [2048]: a pass's pair words, then its ids (16-byte aligned)
    uint32_t* cur = s_id + kThreads * kColItems;       // [TX]
    uint32_t* boff = cur + TX;                         // [TX]
    uint32_t* s_off = boff + TX;                       // [kPlRound]: start of each covering rank's run
    uint16_t* wcnt = reinterpret_cast<uint16_t*>(s_off + kPlRound);   // [kWaves][TX] (a pass has <= 2048 pairs)
    uint16_t* s_x = wcnt + kWaves * TX;                // [2048]
    uint16_t* s_x0 = s_x + kThreads * kColItems;       // [kPlRound]: its first tile
    uint16_t* s_rk = s_x0 + kPlRound;                  // [kPlRound]: its rank within the round
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t wcov[kWaves];
    // workgroups go to the 8 XCDs round-robin by linear id: block b runs on XCD
    // b % 8, and XCD x takes the groups x, x + 8, ... with all their rows, so a
    // group's rects, ids and offsets are read through one XCD's L2
    const int xcd = (int)(blockIdx.x & 7u), m = (int)(blockIdx.x >> 3), v = blockIdx.y;
    const int j = m / B.tiles_y, y = m - j * B.tiles_y, g = xcd + 8 * j;
    if (g >= B.G) return;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t n = *n_pairs;
    const bool fits = n >= 0 && n <= capacity;
    const int64_t vy = (int64_t)v * B.tiles_y + y;
    if (g == 0) {
        const int64_t rb = rbase[vy];
        for (int x = threadIdx.x; x < TX; x += kThreads) {
            const int64_t i = (int64_t)v * B.T + (int64_t)y * TX + x;
            const int64_t b = rb + trel[i], e = rb + (x + 1 < TX ? trel[i + 1] : rtot[vy]);
            const bool any = fits && e > b;
            ranges[2 * i] = any ? (int32_t)b : 0;
            ranges[2 * i + 1] = any ? (int32_t)e : 0;
        }
    }
    if (!fits) return;
    const uint32_t len = gsum[vy * B.G + g];   // the group's pairs in the row
    if (len == 0) return;
    const uint32_t* orow = off + ((int64_t)v * B.G + g) * B.T + (int64_t)y * TX;
    const uint32_t* gorder = order + (int64_t)v * B.N + (int64_t)g * kGroupRanks;
    const uint2* grect = srect + (int64_t)v * B.N + (int64_t)g * kGroupRanks;
    for (int x = threadIdx.x; x < TX; x += kThreads) cur[x] = orow[x];
    const int ns = (int)min((int64_t)kGroupRanks, B.N - (int64_t)g * kGroupRanks);
    const int per = (TX + kThreads - 1) / kThreads;   // counters per thread in the block scan
    uint32_t placed = 0, expanded = 0, fill = 0;
    // one pass over the pair words s_id[0, cntb): rank by tile x, sort in LDS,
    // store each tile's run at its cursor and advance the cursors
    auto place_pass = [&](const uint32_t cntb) {
        for (int t = threadIdx.x; t < kWaves * TX; t += kThreads) wcnt[t] = 0;
        __syncthreads();
        uint32_t key[kColItems], val[kColItems], rnk[kColItems];
#pragma unroll
        for (int k = 0; k < kColItems; ++k) {
            const uint32_t e = (uint32_t)(w * 64 * kColItems + k * 64 + lane);
            key[k] = s_id[min(e, cntb - 1)];
        }
        // all id gathers first, without branches, so that they stay in flight together
#pragma unroll
        for (int k = 0; k < kColItems; ++k) {
            val[k] = gorder[key[k] & (kGroupRanks - 1)];   // the splat id
            key[k] >>= kRankBits;
        }
        // slots of this wave that hold pairs of the pass (the rest are skipped)
        const uint32_t wb0 = (uint32_t)(w * 64 * kColItems);
        const int kn = cntb > wb0 ? (int)min((uint32_t)kColItems, (cntb - wb0 + 63) / 64) : 0;
#pragma unroll
        for (int k = 0; k < kColItems; ++k) {
            if (k >= kn) {
                rnk[k] = 0xffffffffu;
                continue;
            }
            const uint32_t e = (uint32_t)(w * 64 * kColItems + k * 64 + lane);
            const bool ok = e < cntb;
            const uint32_t d = ok ? key[k] : 0u;
            key[k] = d;
            uint32_t below, c;
            match_rank<XBITS>(d, ok, below, c);
            uint32_t r = 0;
            if (ok) r = wcnt[w * TX + d];
            __builtin_amdgcn_wave_barrier();
            if (ok && below == 0) wcnt[w * TX + d] = (uint16_t)(r + c);
            __builtin_amdgcn_wave_barrier();
            rnk[k] = ok ? r + below : 0xffffffffu;
        }
        __syncthreads();
        // per x: exclusive prefix over waves, block count; then the block scan of the counts
        uint32_t local[8];
        uint32_t mine = 0;
        for (int j = 0; j < per; ++j) {
            const int x = threadIdx.x * per + j;
            uint32_t run = 0;
            if (x < TX)
                for (int ww = 0; ww < kWaves; ++ww) {
                    const uint32_t c = wcnt[ww * TX + x];
                    wcnt[ww * TX + x] = (uint16_t)run;
                    run += c;
                }
            local[j] = run;
            mine += run;
        }
        uint32_t pre = block_excl_scan<kThreads>(mine, wsum);
        for (int j = 0; j < per; ++j) {
            const int x = threadIdx.x * per + j;
            if (x < TX) boff[x] = pre;
            pre += local[j];
        }
        __syncthreads();
#pragma unroll
        for (int k = 0; k < kColItems; ++k) {
            if (rnk[k] == 0xffffffffu) continue;
            const uint32_t p = boff[key[k]] + wcnt[w * TX + key[k]] + rnk[k];
            s_id[p] = val[k];
            s_x[p] = (uint16_t)key[k];
        }
        __syncthreads();
        for (uint32_t i = threadIdx.x; i < cntb; i += kThreads) {
            const uint32_t x = s_x[i];
            ids[cur[x] + (i - boff[x])] = s_id[i];
        }
        __syncthreads();
        // advance the cursors past this pass's runs
        for (int x = threadIdx.x; x < TX; x += kThreads) {
            const uint32_t end = (x + 1 < TX) ? boff[x + 1] : cntb;
            cur[x] += end - boff[x];
        }
        __syncthreads();
    };
    for (int h0 = 0; h0 < ns; h0 += kPlRound) {
        const int nh = min(kPlRound, ns - h0);
        // lane l of wave w holds the round's ranks 512 w + 64 k + l (k < kPlSlots)
        uint32_t wd[kPlSlots], x0v[kPlSlots];
#pragma unroll
        for (int k = 0; k < kPlSlots; ++k) {
            const int rk = w * 64 * kPlSlots + k * 64 + lane;
            const uint2 rr = grect[h0 + min(rk, nh - 1)];
            const uint32_t x0 = rr.x & 0xffffu, x1 = rr.x >> 16;
            const int y0 = (int)(rr.y & 0xffffu), y1 = (int)(rr.y >> 16);
            wd[k] = (rk < nh && y0 <= y && y < y1 && x0 < x1) ? x1 - x0 : 0u;
            x0v[k] = x0;
        }
        // exclusive scans in rank order (slot-major in a wave, then waves): of
        // the widths (run starts) and of the cover flags (places in the list)
        uint32_t carry = 0, ccnt = 0, ofs[kPlSlots], pos[kPlSlots];
#pragma unroll
        for (int k = 0; k < kPlSlots; ++k) {
            const uint32_t inc = wave_incl_scan(wd[k]);
            ofs[k] = carry + inc - wd[k];
            carry += (uint32_t)__builtin_amdgcn_readlane((int32_t)inc, 63);
            const uint64_t cb = __ballot(wd[k] != 0u);
            pos[k] = ccnt + __builtin_amdgcn_mbcnt_hi((uint32_t)(cb >> 32), __builtin_amdgcn_mbcnt_lo((uint32_t)cb, 0u));
            ccnt += (uint32_t)__popcll(cb);
        }
        if (lane == 0) {
            wsum[w] = carry;
            wcov[w] = ccnt;
        }
        __syncthreads();
        uint32_t wb = 0, tot = 0, cb0 = 0, call = 0;
#pragma unroll
        for (int k = 0; k < kWaves; ++k) {
            if (k < w) {
                wb += wsum[k];
                cb0 += wcov[k];
            }
            tot += wsum[k];
            call += wcov[k];
        }
        const int ncov = (int)call;   // covering ranks of the round; tot: their pairs
#pragma unroll
        for (int k = 0; k < kPlSlots; ++k) {
            if (wd[k] != 0u) {
                const uint32_t idx = cb0 + pos[k];
                s_off[idx] = wb + ofs[k];
                s_x0[idx] = (uint16_t)x0v[k];
                s_rk[idx] = (uint16_t)(w * 64 * kPlSlots + k * 64 + lane);
            }
        }
        __syncthreads();
        if (placed + tot > len) return;   // cannot happen: the counts come from the same rects
        placed += tot;
        // expand the round's pairs into the pass buffer behind those already there
        for (uint32_t q0 = 0; q0 < tot;) {
            const uint32_t take = min(tot - q0, (uint32_t)(kThreads * kColItems) - fill);
            // this thread fills the buffer slots b0 .. b0 + kPlPer - 1 that this expansion reaches
            const uint32_t b0 = threadIdx.x * kPlPer;
            const uint32_t blo = max(b0, fill), bhi = min(b0 + kPlPer, fill + take);
            if (blo < bhi) {
                const uint32_t qa = q0 + (blo - fill);
                int lo = 0, hi = ncov - 1;   // last run starting at or before qa
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (s_off[mid] <= qa) lo = mid;
                    else hi = mid - 1;
                }
                int r = lo;
                uint32_t o = s_off[r], end = r + 1 < ncov ? s_off[r + 1] : tot;
                uint32_t wv[kPlPer];
#pragma unroll
                for (int i = 0; i < kPlPer; ++i) {
                    const uint32_t b = b0 + i;
                    wv[i] = 0u;
                    if (b >= blo && b < bhi) {
                        const uint32_t q = q0 + (b - fill);
                        if (q >= end) {   // runs are never empty: q is in the next one
                            ++r;
                            o = end;
                            end = r + 1 < ncov ? s_off[r + 1] : tot;
                        }
                        wv[i] = (((uint32_t)s_x0[r] + (q - o)) << kRankBits) | (uint32_t)(h0 + s_rk[r]);
                    }
                }
                if (blo == b0 && bhi == b0 + kPlPer) {   // whole slot block: two 16-byte stores
                    uint4* dst = reinterpret_cast<uint4*>(s_id + b0);
                    dst[0] = make_uint4(wv[0], wv[1], wv[2], wv[3]);
                    dst[1] = make_uint4(wv[4], wv[5], wv[6], wv[7]);
                } else {
#pragma unroll
                    for (int i = 0; i < kPlPer; ++i)
                        if (b0 + i >= blo && b0 + i < bhi) s_id[b0 + i] = wv[i];
                }
            }
            fill += take;
            q0 += take;
            expanded += take;
            if (fill == (uint32_t)(kThreads * kColItems) || expanded == len) {
                place_pass(fill);
                fill = 0;
            }
        }
        __syncthreads();   // the next round rewrites wsum and the run offsets
    }
}

// ---------------------------------------------------------------- host side
// Region at the front of the workspace, cleared at the start of every bin:
// tickets (one per depth pass), the fault word, digit totals, the key range and
// the look-back status words.
struct Ctl {
    uint32_t* ticket;
    uint32_t* fault;
    uint32_t* ghist;
    uint32_t* krange;   // per view: largest key, largest complemented key
    uint64_t* status;
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
    uint32_t *gsum, *rtot;
    int64_t* rbase;
    uint32_t *tc, *toff, *segt, *trel;
    size_t bytes;
};

BinWs bin_layout(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y, char* base) {
    const int64_t VN = N * V;
    const int64_t bps = ceil_div(N > 0 ? N : 1, kTile);
    const Bins B = bins_of(N, V, tiles_x, tiles_y);
    BinWs w;
    size_t o = 0;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b > 0 ? b : 1); return p; };
    // a ticket per depth pass, the tile-row counter of k_tile_bases, the fault word
    w.ctl.ticket = (uint32_t*)take(4 * (kMaxPasses + 2));
    w.ctl.fault = w.ctl.ticket + kMaxPasses + 1;
    w.ctl.ghist = (uint32_t*)take(4 * (size_t)V * kMaxPasses * 256);
    w.ctl.krange = (uint32_t*)take(4 * 2 * (size_t)V);
    w.ctl.status = (uint64_t*)take(8 * (size_t)V * bps * 256);
    const size_t ty = (size_t)tiles_y, T = (size_t)B.T;
    // cleared with the control words: the sums the group counts add into
    w.segt = (uint32_t*)take(4 * (size_t)V * B.nseg_g * T);
    w.ctl.clear_words = (int64_t)(o / 8);
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
    w.bytes = o;
    return w;
}


potr_status sweep(const uint32_t* kin, uint32_t* kout, const uint32_t* vin, uint32_t* vout, uint32_t* vfinal,
                  const Seg& g, int segs, const Pass& P, const uint32_t* krange, hipStream_t s) {
    hipLaunchKernelGGL(k_sweep, dim3((unsigned)((int64_t)g.bps * segs)), dim3(kSwThreads), 0, s, kin, kout, vin, vout,
                       vfinal, g, P, krange);
    return check_launch("k_sweep");
}

// rows per band of the group counts' difference array, and its LDS bytes
int gc_band(int tiles_x) {
    const int rows = (int)(kGcLds / (4 * (size_t)(tiles_x + 1))) - 1;
    return std::max(1, std::min(kGcBand, rows));
}
size_t gc_lds(int band, int tiles_x) { return (size_t)(band + 1) * (tiles_x + 1) * 4; }

// LDS of the placement: cursors and bases per tile, a pass of pair words / ids,
// a round's run starts, 16-bit per-wave counters per tile, a pass's tile x, and
// a round's first tiles and ranks (54 KB at 1600 tile columns)
size_t place_lds(const Bins& B) {
    return ((size_t)2 * B.tiles_x + (size_t)kThreads * kColItems + kPlRound) * 4 +
           ((size_t)kWaves * B.tiles_x + (size_t)kThreads * kColItems + 2 * kPlRound) * 2;
}


}  // namespace

size_t bin_workspace_bytes(int64_t N, int32_t V, int32_t tiles_x, int32_t tiles_y) {
    return bin_layout(N, V, tiles_x, tiles_y, nullptr).bytes;
}

// The placement stages nothing in global memory; the workspace stays in the ABI
// as a placeholder of one aligned block.
size_t sort_workspace_bytes(int64_t) { return align_up(256); }

potr_status launch_bin(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                       const potr_proj* proj, void* ws, uint32_t* order, int64_t* n_pairs, hipStream_t s) {
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
        hipLaunchKernelGGL(k_keys, kg, dim3(kHistThreads), 0, s, proj, N, w.ka, w.crect, w.ctl.krange);
        st = check_launch("k_keys");
        if (st != POTR_OK) return st;
        hipLaunchKernelGGL(k_digits, kg, dim3(kHistThreads), 0, s, (const uint32_t*)w.ka, N,
                           (const uint32_t*)w.ctl.krange, w.ctl.ghist);
        st = check_launch("k_digits");
        if (st != POTR_OK) return st;
        uint32_t *kin = w.ka, *kout = w.kb;
        const uint32_t* vin = nullptr;
        uint32_t* vbuf[2] = {w.va, w.vb};   // never the output: a view's last pass may be any of them
        for (int pass = 0; pass < kMaxPasses; ++pass) {
            Pass P{pass, 8 * pass, 8, (uint32_t)(1 + pass), w.ctl.ghist + pass * 256, w.ctl.status,
                   w.ctl.ticket + pass, w.ctl.fault};
            st = sweep(kin, kout, vin, vbuf[pass & 1], order, g, V, P, w.ctl.krange, s);
            if (st != POTR_OK) return st;
            vin = vbuf[pass & 1];
            uint32_t* t = kin;
            kin = kout;
            kout = t;
        }
        const int band = gc_band(txs);
        hipLaunchKernelGGL(k_count, dim3(B.G, V), dim3(kGcThreads), gc_lds(band, txs), s, (const uint32_t*)order,
                           (const uint2*)w.crect, B, band, w.srect, w.gsum, w.tc, w.segt);
        st = check_launch("k_count");
        if (st != POTR_OK) return st;
    }
    // tile starts within their rows and row totals, then row bases over
    // (view, row), the pair count, and every group's first position per tile
    hipLaunchKernelGGL(k_tile_bases, dim3(tys, V), dim3(256), 0, s, w.segt, B, w.trel, w.rtot, w.ctl.ticket + kMaxPasses,
                       (const uint32_t*)w.ctl.fault, w.rbase, n_pairs);
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
    (void)sort_ws;   // nothing is staged in global memory
    if (N == 0) {
        // no pairs: every tile range is [0, 0)
        const int64_t words = (int64_t)V * B.T;
        hipLaunchKernelGGL(k_clear, dim3((unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(words, 256), 4096))),
                           dim3(256), 0, s, (uint64_t*)tile_ranges, words);
        return check_launch("k_clear");
    }
    // every (group, row) segment to its tiles (and the tile ranges)
    const dim3 gp((unsigned)(8 * ceil_div(B.G, 8) * tys), V);   // see the XCD mapping in k_place
    const size_t lds = place_lds(B);
    const uint2* sr = w.srect;
    const uint32_t* gs = w.gsum;
    const uint32_t* to = w.toff;
    const int64_t* rb = w.rbase;
    const uint32_t* tr = w.trel;
    const uint32_t* rt = w.rtot;
    switch (B.xbits) {
        case 1: case 2: case 3: case 4: case 5:
            hipLaunchKernelGGL(k_place<5>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        case 6:
            hipLaunchKernelGGL(k_place<6>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        case 7:
            hipLaunchKernelGGL(k_place<7>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        case 8:
            hipLaunchKernelGGL(k_place<8>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        case 9:
            hipLaunchKernelGGL(k_place<9>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        case 10:
            hipLaunchKernelGGL(k_place<10>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
        default:
            hipLaunchKernelGGL(k_place<11>, gp, dim3(kThreads), lds, s, sr, gs, to, rb, tr, rt, B, n_pairs, capacity, order,
                               sorted_ids, tile_ranges);
            break;
    }
    return check_launch("k_place");
}

}  // namespace potr
