// Depth ordering and tile binning (paper Sec. 3: splats composited in layers
// ordered by approximate depth), as stable LSD radix sorts.
//
// potr_bin: per view, a stable radix sort of the N depth keys (ties keep splat
//   id order) gives each splat its depth rank; the pairs (tile, splat id) of
//   every splat's rect are then emitted in rank order, each splat's run placed
//   by a scan of tiles_touched in rank order.
// potr_sort: a stable radix sort of the pairs on the (view, tile) bits only.
//   Pairs were emitted in depth-rank order and the sort is stable, so the
//   result is ordered by (view, tile, depth key, splat id) -- the full key --
//   while only ceil(log2(V * tiles)) bits are sorted instead of tile + 32 depth
//   bits. The low bits carry the splat id as payload.
//
// Pairs are packed as ((view * tiles + tile) << id_bits) | splat id in 32 bits
// when both fields fit, else in 64 bits with the id in the low word.
//
// Every radix pass is one kernel: a block of 256 threads x 16 items ranks its
// keys per digit with 64-lane ballots (stable order: wave, item, lane),
// publishes its digit counts, and finds the counts of all blocks before it by
// decoupled look-back over their published words. The digit totals of all
// passes come from one histogram read up front. Blocks take their place in the
// chain from an atomic ticket, so a block only ever waits on blocks that are
// already running. Each block sorts its keys in LDS and writes every digit's
// run to consecutive addresses.
//
// Every wait is bounded: after kSpinLimit polls the block records a fault and
// goes on (the results are then wrong and the bin reports n_pairs = -1), so no
// input can leave a kernel spinning.
#include <algorithm>

#include "common.h"

namespace potr {
namespace {

constexpr int kThreads = 256;
constexpr int kItems = 16;
constexpr int kTile = kThreads * kItems;     // keys per block
constexpr int kWaves = kThreads / 64;
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
// adds aggregates walking back until an inclusive prefix is found.
__device__ uint64_t look_back_serial(uint64_t* st, int64_t b, int stride, uint32_t tag, uint32_t* fault) {
    uint64_t excl = 0;
    uint32_t spins = 0;
    for (int64_t p = b - 1; p >= 0;) {
        const uint64_t w = st_get(st + p * stride);
        const uint32_t s = st_state(w, tag);
        if (s == 0) {
            if (++spins > kSpinLimit) {
                atomicOr(fault, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += w & kValMask;
        if (s == kStInc) break;
        --p;
    }
    return excl;
}

__device__ inline int64_t wave_sum_i64(int64_t v) {
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// Same, one wave polling 64 predecessors at a time (call with the whole wave).
__device__ int64_t look_back_wave(uint64_t* st, int64_t b, uint32_t tag, uint32_t* fault) {
    const int lane = threadIdx.x & 63;
    int64_t excl = 0;
    int64_t hi = b - 1;
    uint32_t spins = 0;
    while (hi >= 0) {
        const int64_t p = hi - lane;
        uint64_t w = 0;
        uint32_t s = (uint32_t)kStInc;     // before block 0: an inclusive zero
        if (p >= 0) {
            w = st_get(st + p);
            s = st_state(w, tag);
        }
        const uint64_t inc = __ballot(s == kStInc);
        const uint64_t none = __ballot(s == 0);
        const uint64_t upto = inc ? ((inc & (~inc + 1)) << 1) - 1 : ~0ull;   // lanes up to the nearest inclusive
        if (none & upto) {
            if (++spins > kSpinLimit) {
                if (lane == 0) atomicOr(fault, 1u);
                break;
            }
            __builtin_amdgcn_s_sleep(1);
            continue;
        }
        excl += wave_sum_i64(((upto >> lane) & 1ull) ? (int64_t)(w & kValMask) : 0);
        if (inc) break;
        hi -= 64;
    }
    return excl;
}

// Exclusive scan of one value per thread over the block (256 threads).
__device__ inline uint32_t block_excl_scan(uint32_t x, uint32_t* wsum) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    uint32_t inc = x;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) wsum[w] = inc;
    __syncthreads();
    uint32_t pre = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k)
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
    int32_t shift, bits;
    uint32_t tag;             // 1 + pass index
    const uint32_t* ghist;    // this pass's digit totals at ghist[seg * kMaxPasses * 256 + digit]
    uint64_t* status;         // [seg][bps][1 << bits]
    uint32_t* ticket;
    uint32_t* fault;
};

// Digit totals of every pass for each segment, in one read of the keys. With
// proj != nullptr the keys are the depth bits of the records and are written
// to keys_out on the way.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_hist(const K* __restrict__ keys, const potr_proj* __restrict__ proj,
                                                   uint32_t* __restrict__ keys_out, Seg g, int n_passes,
                                                   int shift0, int per, int bits_total, uint32_t* __restrict__ ghist) {
    __shared__ uint32_t h[kMaxPasses][256];
    for (int t = threadIdx.x; t < kMaxPasses * 256; t += kThreads) (&h[0][0])[t] = 0;
    __syncthreads();
    const int seg = blockIdx.y;
    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.len;
    for (int64_t e = (int64_t)blockIdx.x * kThreads + threadIdx.x; e < n; e += (int64_t)gridDim.x * kThreads) {
        K k;
        if (proj) {
            k = (K)__float_as_uint(proj[seg0 + e].depth);
            keys_out[seg0 + e] = (uint32_t)k;
        } else {
            k = keys[seg0 + e];
        }
        for (int p = 0; p < n_passes; ++p) {
            const int b = (p == n_passes - 1) ? bits_total - per * p : per;
            atomicAdd(&h[p][digit_of(k, shift0 + per * p, (1u << b) - 1)], 1u);
        }
    }
    __syncthreads();
    for (int t = threadIdx.x; t < n_passes * 256; t += kThreads) {
        const uint32_t c = (&h[0][0])[t];
        if (c) atomicAdd(ghist + (int64_t)seg * kMaxPasses * 256 + t, c);
    }
}

// Outputs of the last pass over the pairs: the splat ids, and each tile's
// range from atomic min / max over the positions where a block's run of that
// tile starts and ends (a tile's pairs are contiguous in every block and
// globally, so these are its global first and last positions).
struct Final {
    uint32_t* ids;
    int32_t* ranges;
    int32_t gshift;          // key >> gshift = view * tiles + tile
    uint64_t imask;          // key & imask = splat id
};

// One stable radix pass. MODE 0: keys and values (values from vin, or the
// element's index when vin == nullptr); MODE 1: keys only; MODE 2 (last depth
// pass): only the values go out, to vout, with cnt_out[pos] = tt[value];
// MODE 3 (last pair pass): ids and tile ranges (Final) instead of keys.
template <typename K, int MODE>
__global__ __launch_bounds__(kThreads) void k_sweep(const K* __restrict__ kin, K* __restrict__ kout,
                                                    const uint32_t* __restrict__ vin, uint32_t* __restrict__ vout,
                                                    Seg g, Pass P, const int32_t* __restrict__ tt,
                                                    int32_t* __restrict__ cnt_out, Final F) {
    constexpr bool VALS = MODE == 0 || MODE == 2;
    __shared__ uint32_t wcnt[kWaves][256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t boff[256];
    __shared__ uint32_t wsum[kWaves];
    __shared__ uint32_t s_ticket;
    __shared__ K s_key[kTile];
    __shared__ uint32_t s_val[VALS ? kTile : 1];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint32_t radix = 1u << P.bits, mask = radix - 1;
    if (threadIdx.x == 0) s_ticket = atomicAdd(P.ticket, 1u);
    for (int t = threadIdx.x; t < kWaves * 256; t += kThreads) (&wcnt[0][0])[t] = 0;
    __syncthreads();
    const int seg = (int)(s_ticket / (uint32_t)g.bps);
    const int64_t b = (int64_t)(s_ticket - (uint32_t)seg * (uint32_t)g.bps);
    const int64_t n = seg_n(g);
    const int64_t seg0 = (int64_t)seg * g.len;
    const int64_t blk0 = b * kTile;
    const int64_t wbase = blk0 + (int64_t)w * (64 * kItems);

    // this segment's digit bases: exclusive scan of the pass's digit totals
    const uint32_t gh = threadIdx.x < radix ? P.ghist[(int64_t)seg * kMaxPasses * 256 + threadIdx.x] : 0u;
    const uint32_t dbase = block_excl_scan(gh, wsum);

    K key[kItems];
    uint32_t val[kItems];
    uint32_t rnk[kItems];
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        const int64_t e = wbase + k * 64 + lane;
        const bool ok = e < n;
        key[k] = ok ? kin[seg0 + e] : (K)0;
        if (VALS) val[k] = ok ? (vin ? vin[seg0 + e] : (uint32_t)e) : 0u;
        const uint32_t d = digit_of(key[k], P.shift, mask);
        uint64_t m = __ballot(ok);
        for (int bit = 0; bit < P.bits; ++bit) {
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
    // per digit: exclusive prefix over waves (waves hold consecutive runs) and the block count
    uint32_t run = 0;
    if (threadIdx.x < radix) {
        const uint32_t d = threadIdx.x;
#pragma unroll
        for (int ww = 0; ww < kWaves; ++ww) {
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
            excl = look_back_serial(st, b, (int)radix, P.tag, P.fault);
            st_put(st + b * radix, st_word(P.tag, kStInc, excl + run));
        }
        goff[d] = dbase + (uint32_t)excl;
    }
    // exclusive scan of the block's digit counts: LDS position of each digit's run
    boff[threadIdx.x] = block_excl_scan(run, wsum);
    __syncthreads();
    // block-local sort in LDS
#pragma unroll
    for (int k = 0; k < kItems; ++k) {
        if (rnk[k] == 0xffffffffu) continue;
        const uint32_t d = digit_of(key[k], P.shift, mask);
        const uint32_t p = boff[d] + wcnt[w][d] + rnk[k];
        s_key[p] = key[k];
        if (VALS) s_val[p] = val[k];
    }
    __syncthreads();
    // coalesced write-out: digit runs go to consecutive global addresses
    const int64_t left = n - blk0;
    const int cnt_blk = left < kTile ? (int)(left > 0 ? left : 0) : kTile;
    for (int i = threadIdx.x; i < cnt_blk; i += kThreads) {
        const K kk = s_key[i];
        const uint32_t d = digit_of(kk, P.shift, mask);
        const int64_t pos = seg0 + (int64_t)goff[d] + (i - (int)boff[d]);
        if (MODE == 0 || MODE == 1) kout[pos] = kk;
        if (MODE == 0) vout[pos] = s_val[i];
        if (MODE == 2) {
            const uint32_t id = s_val[i];
            vout[pos] = id;
            cnt_out[pos] = tt[seg0 + id];
        }
        if (MODE == 3) {
            F.ids[pos] = (uint32_t)((uint64_t)kk & F.imask);
            const uint32_t gi = (uint32_t)((uint64_t)kk >> F.gshift);
            if (i == 0 || (uint32_t)((uint64_t)s_key[i - 1] >> F.gshift) != gi)
                atomicMin(F.ranges + 2 * (int64_t)gi, (int32_t)pos);
            if (i == cnt_blk - 1 || (uint32_t)((uint64_t)s_key[i + 1] >> F.gshift) != gi)
                atomicMax(F.ranges + 2 * (int64_t)gi + 1, (int32_t)pos + 1);
        }
    }
}

// ---------------------------------------------------------------- bin kernels
// Clears 64-bit words (look-back status, digit totals, tickets).
__global__ void k_clear(uint64_t* __restrict__ p, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        p[i] = 0;
}

// Tile ranges before the last pass: start = INT32_MAX (for atomic min), end = 0.
__global__ void k_ranges_init(int32_t* r, int64_t n_tiles, int32_t start) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles;
         t += (int64_t)gridDim.x * blockDim.x) {
        r[2 * t] = start;
        r[2 * t + 1] = 0;
    }
}

// Tiles no pair reached get the empty range [0, 0).
__global__ void k_ranges_fix(int32_t* r, int64_t n_tiles) {
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n_tiles;
         t += (int64_t)gridDim.x * blockDim.x)
        if (r[2 * t] == INT32_MAX) r[2 * t] = 0;
}

// Pairs of 256 consecutive (view, rank) entries per block. The pair offset of
// the block comes from a decoupled look-back over the blocks before it; each
// wave then writes its 64 splats' runs one splat at a time, lanes covering
// consecutive tiles of the rect, so stores are contiguous.
template <typename K>
__global__ __launch_bounds__(kThreads) void k_emit(const uint32_t* __restrict__ order, const int32_t* __restrict__ cnt,
                                                   const potr_proj* __restrict__ proj, int64_t N, int64_t total,
                                                   int32_t tiles_x, int32_t tiles_per_view, int id_bits,
                                                   int64_t capacity, uint64_t* status, uint32_t* ticket,
                                                   uint32_t* fault, int64_t n_blocks, int64_t* __restrict__ n_pairs,
                                                   K* __restrict__ pairs) {
    __shared__ uint32_t s_ticket;
    __shared__ int64_t s_wsum[kWaves];
    __shared__ int64_t s_excl;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    if (threadIdx.x == 0) s_ticket = atomicAdd(ticket, 1u);
    __syncthreads();
    const int64_t b = s_ticket;
    const int64_t i = b * kThreads + threadIdx.x;
    int64_t c = 0;
    uint32_t id = 0, g0 = 0, wdt = 1;
    if (i < total) {
        const int32_t ci = cnt[i];
        if (ci > 0) {
            const int64_t v = i / N;
            id = order[i];
            const potr_proj& p = proj[v * N + id];
            c = ci;
            g0 = (uint32_t)(v * tiles_per_view + p.rect[1] * tiles_x + p.rect[0]);
            wdt = (uint32_t)(p.rect[2] - p.rect[0]);
        }
    }
    int64_t inc = c;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int64_t y = __shfl_up(inc, d, 64);
        if (lane >= d) inc += y;
    }
    if (lane == 63) s_wsum[wid] = inc;
    __syncthreads();
    int64_t pre = 0, sum = 0;
#pragma unroll
    for (int k = 0; k < kWaves; ++k) {
        if (k < wid) pre += s_wsum[k];
        sum += s_wsum[k];
    }
    if (wid == 0) {
        int64_t excl = 0;
        if (b == 0) {
            if (lane == 0) st_put(status, st_word(1, kStInc, (uint64_t)sum));
        } else {
            if (lane == 0) st_put(status + b, st_word(1, kStAgg, (uint64_t)sum));
            excl = look_back_wave(status, b, 1, fault);
            if (lane == 0) st_put(status + b, st_word(1, kStInc, (uint64_t)(excl + sum)));
        }
        if (lane == 0) {
            s_excl = excl;
            if (b == n_blocks - 1)
                *n_pairs = __hip_atomic_load(fault, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ? (int64_t)-1
                                                                                                : excl + sum;
        }
    }
    __syncthreads();
    const int64_t start = s_excl + pre + inc - c;
    for (int s = 0; s < 64; ++s) {
        const int32_t cs = __builtin_amdgcn_readlane((int32_t)c, s);
        if (cs == 0) continue;
        const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)start, s);
        const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int32_t)(uint32_t)((uint64_t)start >> 32), s);
        const int64_t st = (int64_t)(((uint64_t)hi << 32) | lo);
        const uint32_t sid = (uint32_t)__builtin_amdgcn_readlane((int32_t)id, s);
        const uint32_t sg0 = (uint32_t)__builtin_amdgcn_readlane((int32_t)g0, s);
        const int32_t sw = __builtin_amdgcn_readlane((int32_t)wdt, s);
        const float rw = 1.0f / (float)sw;
        for (int32_t k = lane; k < cs; k += 64) {
            // tile k of the rect, row-major: k = ty * width + tx (the float
            // quotient is off by at most one; rows < 2^15)
            int32_t ty = (int32_t)((float)k * rw);
            int32_t tx = k - ty * sw;
            if (tx < 0) {
                --ty;
                tx += sw;
            } else if (tx >= sw) {
                ++ty;
                tx -= sw;
            }
            const int64_t p = st + k;
            if (p < capacity) {
                const uint64_t gg = (uint64_t)sg0 + (uint64_t)ty * (uint32_t)tiles_x + (uint32_t)tx;
                if (sizeof(K) == 4)
                    pairs[p] = (K)((gg << id_bits) | sid);
                else
                    pairs[p] = (K)((gg << 32) | sid);
            }
        }
    }
}

// ---------------------------------------------------------------- host side
int bit_width(int64_t x) {           // bits to hold 0..x (at least 1)
    int b = 1;
    while (b < 62 && (int64_t(1) << b) <= x) ++b;
    return b;
}

struct Packing {
    int tile_bits, id_bits;
    bool u32;
};

Packing packing(int64_t N, int32_t V, int32_t tiles_per_view) {
    Packing p;
    p.tile_bits = bit_width((int64_t)V * tiles_per_view - 1);
    p.id_bits = bit_width(N > 0 ? N - 1 : 0);
    p.u32 = p.tile_bits + p.id_bits <= 32;
    return p;
}

// Region at the front of each workspace, cleared at the start of every call:
// tickets (one per pass + one for the emit), the fault word, digit totals and
// the look-back status words.
struct Ctl {
    uint32_t* ticket;
    uint32_t* fault;
    uint32_t* ghist;
    uint64_t* status;       // radix passes
    uint64_t* estatus;      // emit (bin only)
    int64_t clear_words;
};

Ctl ctl_layout(char* base, size_t& o, int64_t segs, int64_t status_words, int64_t estatus_words) {
    Ctl c;
    const size_t o0 = o;
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    c.ticket = (uint32_t*)take(4 * (kMaxPasses + 2));
    c.fault = c.ticket + kMaxPasses + 1;
    c.ghist = (uint32_t*)take(4 * (size_t)segs * kMaxPasses * 256);
    c.status = (uint64_t*)take(8 * (size_t)status_words);
    c.estatus = (uint64_t*)take(8 * (size_t)(estatus_words > 0 ? estatus_words : 1));
    c.clear_words = (int64_t)((o - o0) / 8);
    return c;
}

struct BinWs {
    uint32_t *ka, *kb, *va;
    int32_t* cnt;
    Ctl ctl;
    size_t bytes;
};

BinWs bin_layout(int64_t N, int32_t V, char* base) {
    const int64_t VN = N * V;
    const int64_t bps = ceil_div(N > 0 ? N : 1, kTile);
    BinWs w;
    size_t o = 0;
    w.ctl = ctl_layout(base, o, V, (int64_t)V * bps * 256, ceil_div(VN > 0 ? VN : 1, kThreads));
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    w.ka = (uint32_t*)take(4 * VN);
    w.kb = (uint32_t*)take(4 * VN);
    w.va = (uint32_t*)take(4 * VN);
    w.cnt = (int32_t*)take(4 * VN);
    w.bytes = o;
    return w;
}

struct SortWs {
    void* alt;
    Ctl ctl;
    size_t bytes;
};

SortWs sort_layout(int64_t cap, char* base) {
    const int64_t bps = ceil_div(cap > 0 ? cap : 1, kTile);
    SortWs w;
    size_t o = 0;
    w.ctl = ctl_layout(base, o, 1, bps * 256, 0);
    auto take = [&](size_t b) { char* p = base ? base + o : nullptr; o += align_up(b); return p; };
    w.alt = take(8 * (size_t)(cap > 0 ? cap : 1));
    w.bytes = o;
    return w;
}

potr_status clear(const Ctl& c, hipStream_t s) {
    const unsigned blocks = (unsigned)std::min<int64_t>(ceil_div(c.clear_words, 256), 4096);
    hipLaunchKernelGGL(k_clear, dim3(blocks), dim3(256), 0, s, (uint64_t*)c.ticket, c.clear_words);
    return check_launch("k_clear");
}

unsigned hist_blocks(int64_t n, int segs) {
    return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 4 * kThreads), 2048 / segs));
}

template <typename K, int MODE>
potr_status sweep(const K* kin, K* kout, const uint32_t* vin, uint32_t* vout, const Seg& g, int segs, const Pass& P,
                  const int32_t* tt, int32_t* cnt_out, const Final& F, hipStream_t s) {
    hipLaunchKernelGGL((k_sweep<K, MODE>), dim3((unsigned)((int64_t)g.bps * segs)), dim3(kThreads), 0, s, kin, kout,
                       vin, vout, g, P, tt, cnt_out, F);
    return check_launch("k_sweep");
}

unsigned grid_for(int64_t n) { return (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 4096)); }

template <typename K>
potr_status emit_pairs(const uint32_t* order, const BinWs& w, const potr_proj* proj, int64_t N, int64_t VN, int txs,
                       int tpv, int id_bits, int64_t capacity, int64_t* n_pairs, void* pairs, hipStream_t s) {
    const int64_t nb = ceil_div(VN > 0 ? VN : 1, kThreads);
    hipLaunchKernelGGL(k_emit<K>, dim3((unsigned)nb), dim3(kThreads), 0, s, order, (const int32_t*)w.cnt, proj,
                       N > 0 ? N : 1, VN, txs, tpv, id_bits, capacity, w.ctl.estatus, w.ctl.ticket + kMaxPasses,
                       w.ctl.fault, nb, n_pairs, (K*)pairs);
    return check_launch("k_emit");
}

template <typename K>
potr_status sort_pairs(const Packing& pk, int64_t n_tiles, const int64_t* n_pairs, int64_t n_max, void* pairs,
                       const SortWs& w, uint32_t* sorted_ids, int32_t* tile_ranges, hipStream_t s) {
    const int bits = pk.tile_bits;
    const int passes = (bits + 7) / 8;
    const int per = (bits + passes - 1) / passes;
    const int shift0 = sizeof(K) == 4 ? pk.id_bits : 32;
    Seg g{0, n_pairs, n_max, (int32_t)ceil_div(n_max, kTile)};
    potr_status st = clear(w.ctl, s);
    if (st != POTR_OK) return st;
    hipLaunchKernelGGL(k_hist<K>, dim3(hist_blocks(n_max, 1), 1), dim3(kThreads), 0, s, (const K*)pairs, nullptr,
                       nullptr, g, passes, shift0, per, bits, w.ctl.ghist);
    st = check_launch("k_hist");
    if (st != POTR_OK) return st;
    const Final F{sorted_ids, tile_ranges, shift0,
                  sizeof(K) == 4 ? ((1ull << pk.id_bits) - 1) : 0xffffffffull};
    K *kin = (K*)pairs, *kout = (K*)w.alt;
    for (int p = 0; p < passes; ++p) {
        const int b = (p == passes - 1) ? bits - per * p : per;
        Pass P{shift0 + per * p, b, (uint32_t)(1 + p), w.ctl.ghist + p * 256, w.ctl.status, w.ctl.ticket + p,
               w.ctl.fault};
        if (p < passes - 1)
            st = sweep<K, 1>(kin, kout, nullptr, nullptr, g, 1, P, nullptr, nullptr, F, s);
        else
            st = sweep<K, 3>(kin, nullptr, nullptr, nullptr, g, 1, P, nullptr, nullptr, F, s);
        if (st != POTR_OK) return st;
        K* t = kin;
        kin = kout;
        kout = t;
    }
    hipLaunchKernelGGL(k_ranges_fix, dim3(grid_for(n_tiles)), dim3(256), 0, s, tile_ranges, n_tiles);
    return check_launch("k_ranges_fix");
}

}  // namespace

size_t bin_workspace_bytes(int64_t N, int32_t V) { return bin_layout(N, V, nullptr).bytes; }

potr_status launch_bin(int64_t N, int32_t V, const potr_camera& cam0, const potr_config& cfg,
                       const potr_proj* proj, const int32_t* tiles_touched, void* ws, uint32_t* order,
                       uint64_t* pairs, int64_t capacity, int64_t* n_pairs, hipStream_t s) {
    BinWs w = bin_layout(N, V, (char*)ws);
    const int64_t VN = N * V;
    const int txs = tiles_x(cam0, cfg), tpv = txs * tiles_y(cam0, cfg);
    const Packing pk = packing(N, V, tpv);
    potr_status st = clear(w.ctl, s);
    if (st != POTR_OK) return st;
    if (VN > 0) {
        // stable per-view sort of the 32-bit depth keys: four 8-bit passes
        Seg g{N, nullptr, 0, (int32_t)ceil_div(N, kTile)};
        hipLaunchKernelGGL(k_hist<uint32_t>, dim3(hist_blocks(N, V), V), dim3(kThreads), 0, s,
                           (const uint32_t*)nullptr, proj, w.ka, g, 4, 0, 8, 32, w.ctl.ghist);
        st = check_launch("k_hist");
        if (st != POTR_OK) return st;
        uint32_t *kin = w.ka, *kout = w.kb;
        const uint32_t* vin = nullptr;
        uint32_t* vbuf[2] = {w.va, order};
        for (int pass = 0; pass < 4; ++pass) {
            Pass P{8 * pass, 8, (uint32_t)(1 + pass), w.ctl.ghist + pass * 256, w.ctl.status, w.ctl.ticket + pass,
                   w.ctl.fault};
            const Final none{nullptr, nullptr, 0, 0};
            if (pass < 3)
                st = sweep<uint32_t, 0>(kin, kout, vin, vbuf[pass & 1], g, V, P, nullptr, nullptr, none, s);
            else
                st = sweep<uint32_t, 2>(kin, nullptr, vin, order, g, V, P, tiles_touched, w.cnt, none, s);
            if (st != POTR_OK) return st;
            vin = vbuf[pass & 1];
            uint32_t* t = kin;
            kin = kout;
            kout = t;
        }
    }
    // with no splats the emit's single empty block reports zero pairs
    if (pk.u32)
        return emit_pairs<uint32_t>(order, w, proj, N, VN, txs, tpv, pk.id_bits, capacity, n_pairs, pairs, s);
    return emit_pairs<uint64_t>(order, w, proj, N, VN, txs, tpv, pk.id_bits, capacity, n_pairs, pairs, s);
}

size_t sort_workspace_bytes(int64_t capacity, int32_t, int32_t) { return sort_layout(capacity, nullptr).bytes; }

potr_status launch_sort(int64_t N, int32_t V, int32_t tiles_per_view, const int64_t* n_pairs, int64_t n_max,
                        uint64_t* pairs, void* ws, uint32_t* sorted_ids, int32_t* tile_ranges, hipStream_t s) {
    SortWs w = sort_layout(n_max, (char*)ws);
    const int64_t n_tiles = (int64_t)V * tiles_per_view;
    hipLaunchKernelGGL(k_ranges_init, dim3(grid_for(n_tiles)), dim3(256), 0, s, tile_ranges, n_tiles,
                       n_max == 0 ? 0 : INT32_MAX);
    potr_status st = check_launch("k_ranges_init");
    if (st != POTR_OK || n_max == 0) return st;
    const Packing pk = packing(N, V, tiles_per_view);
    if (pk.u32) return sort_pairs<uint32_t>(pk, n_tiles, n_pairs, n_max, pairs, w, sorted_ids, tile_ranges, s);
    return sort_pairs<uint64_t>(pk, n_tiles, n_pairs, n_max, pairs, w, sorted_ids, tile_ranges, s);
}

}  // namespace potr
