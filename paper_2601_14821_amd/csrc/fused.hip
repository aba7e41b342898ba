// Fused forward render + removal pass per tile (paper Sec. 3 compositing and
// Sec. 4.2 pruning difference), in two launch forms:
//   k_render_score            one workgroup per (tile, view) of one call
//   k_render_score_persistent a fixed grid of workgroups that pull (view, tile)
//                             items of many scenes and views from a device
//                             counter until the queue is empty
// Per tile: a blend sweep front to back with early stop gives each pixel's P_K,
// T_final and stop position; the removal sweep then revisits the walked prefix.
// When that prefix fits one LDS batch (the usual case: ~100-200 walked entries
// per tile), the records staged for the blend are reused without a second
// gather. The arithmetic per (pixel, splat) is that of potr_blend / potr_score
// (raster_eval.h): the images are the same bit for bit, the per-splat sums up to
// the order of their float additions.
#include <algorithm>

#include "common.h"
#include "dpp.h"
#include "fused.h"
#include "raster_eval.h"

namespace potr {
namespace {

// One staged splat: a, b and (blue, splat id, reachable tile rows, -) side by
// side, so that a sweep reads all three with one address and immediate offsets
// and no per-entry array besides them is needed.
struct Rec {
    float4 a, b, c;
};
constexpr int kRecWords = sizeof(Rec) / 4;
constexpr int kRowsWord = 10;   // word of a Rec holding the reachable rows
static_assert(sizeof(Rec) == 48 && kRowsWord == 8 + 2, "rows are c.z, after a and b");

struct Smem {
    Rec* rec;
    uint16_t* list;    // [NW][B] per-wave lists of the entries reaching the wave's rows
    uint16_t* hits;    // [NW][B] per-wave lists of the entries some lane of the wave blended
    int* misc;         // [0]: wmax
    float* part;       // [n_out][B] per-entry sums over the waves, n_out = number of per-splat outputs (last, sized by the launch)
};

template <int NT, int TH>
__device__ inline void stage(const potr_proj* __restrict__ pv, const uint32_t* __restrict__ ids, int base, int cnt,
                             const Smem& sm, float qmax, int tile_y0) {
    for (int j = threadIdx.x; j < cnt; j += NT) {
        const uint32_t id = ids[base + j];
        const float4* src = reinterpret_cast<const float4*>(pv + id);
        const float4 r0 = src[0], r1 = src[1], r2 = src[2];
        float4 a, b;
        make_rec(r0, r1, a, b);
        sm.rec[j].a = a;
        sm.rec[j].b = b;
        sm.rec[j].c = make_float4(r2.x, __uint_as_float(id), __uint_as_float(reach_rows(a, b, qmax, tile_y0, TH)), 0.f);
    }
}

// Four consecutive entries of a wave list (i a multiple of 4; entries at or
// past the list's end are junk and must not be used). Every lane reads the same
// words; taking them into scalar registers keeps the loop's tests on them scalar.
__device__ inline void list4(const uint16_t* L, int i, int (&j)[4]) {
    const uint2 q = *reinterpret_cast<const uint2*>(L + i);
    const uint32_t x = __builtin_amdgcn_readfirstlane(q.x), y = __builtin_amdgcn_readfirstlane(q.y);
    j[0] = (int)(x & 0xffffu);
    j[1] = (int)(x >> 16);
    j[2] = (int)(y & 0xffffu);
    j[3] = (int)(y >> 16);
}

// Fixed point (FX): per-splat sums in int64 units of 2^-32, added in integers
// (which commute), so that every run gives the same bits whatever the order of
// the waves' and tiles' additions.
constexpr double kFixedOne = 4294967296.0;   // 2^32
__device__ inline unsigned long long to_fixed(double x) { return (unsigned long long)__double2ll_rn(x * kFixedOne); }

template <int TW, int TH, bool SE, bool FX>
__device__ void render_score_tile(const ViewJob& J, int tile, const potr_config& cfg, const Smem& sm) {
    constexpr int NT = TW * TH;
    const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
    const int tile_y0 = (tile / J.tiles_x) * TH;
    const int px = (tile % J.tiles_x) * TW + (int)(threadIdx.x % TW);
    const int py = tile_y0 + (int)(threadIdx.x / TW);
    // tile rows covered by this wave (wave-uniform, kept in scalar registers)
    const int row_lo = __builtin_amdgcn_readfirstlane((wid * 64) / TW);
    const int row_hi = __builtin_amdgcn_readfirstlane((wid * 64 + 63) / TW);
    const bool inside = px < J.W && py < J.H;
    const float fx = (float)px + 0.5f, fy = (float)py + 0.5f;
    const int beg = J.ranges[2 * tile], end = J.ranges[2 * tile + 1];
    const int B = cfg.lds_batch;
    const float qmax = cfg.q_max, amin = cfg.alpha_min, tmin = cfg.t_min;
    // a min's result is canonical, so the per-entry min against it needs no canonicalisation
    const float amax = fminf(cfg.alpha_max, 1.f);
    const float emin = exp_floor(qmax);
    // SE instantiations serve jobs with and without dSE output
    const bool se = SE && J.scores_se != nullptr;
    const int n_out = (J.scores ? 1 : 0) + (J.importance ? 1 : 0) + (se ? 1 : 0);
    const int o_l1 = 0, o_im = J.scores ? 1 : 0, o_se = o_im + (J.importance ? 1 : 0);
    uint16_t* const L = sm.list + wid * B;
    uint16_t* const Hl = sm.hits + wid * B;

    // ---- blend sweep: each wave walks its own list of the batch; the steps
    // are branch-free (a finished lane evaluates alpha = 0, which leaves T and
    // the colour unchanged bit for bit)
    float T = 1.f, cr = 0.f, cg = 0.f, cb = 0.f;
    bool done = !inside;
    int walk = 0;
    int staged = -1;   // list offset of the batch now in LDS
    int nl = 0;        // length of this wave's list for that batch
    int nh = 0;        // length of this wave's list of blended entries for that batch
    for (int base = beg; base < end; base += B) {
        if (__syncthreads_count(!done) == 0) break;
        const int cnt = min(B, end - base);
        const int wofs = __builtin_amdgcn_readfirstlane(base - beg);   // list offset of the batch
        stage<NT, TH>(J.proj, J.ids, base, cnt, sm, qmax, tile_y0);
        staged = base;
        __syncthreads();
        nl = __builtin_amdgcn_readfirstlane(
            wave_list<kRecWords>(reinterpret_cast<const uint32_t*>(sm.rec) + kRowsWord, cnt, row_lo, row_hi, L));
        nh = 0;
        if (__ballot(!done) == 0) continue;
        for (int i = 0; i < nl; i += 4) {
            int js[4];
            list4(L, i, js);
            // the group's records, read before any of them is used (slots past
            // the list's end read entry js[0] and are skipped)
            const int nv = min(4, nl - i);
            float4 ra[4], rb[4];
            float rc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jj = u < nv ? js[u] : js[0];
                ra[u] = sm.rec[jj].a;
                rb[u] = sm.rec[jj].b;
                rc[u] = sm.rec[jj].c.x;
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (u >= nv) break;
                const int j = js[u];
                const float4 b = rb[u];
                const float a0 = alpha_of(eval_gauss(ra[u], b, fx, fy), emin, amin, amax);
                const float al = done ? 0.f : a0;
                float Tn = next_T(T, al);
                const bool stop = Tn < tmin;       // T >= tmin before, so only when al > 0
                float w = __fmul_rn(T, al);
                // a lane stops once per tile: only entries where some lane of the
                // wave stops take the selects (the lane keeps T and adds nothing)
                if (__ballot(stop) != 0) {
                    w = stop ? 0.f : w;
                    Tn = stop ? T : Tn;
                    walk = stop ? wofs + j : walk;
                    done = done || stop;
                }
                cr = add_weighted(cr, w, b.z);
                cg = add_weighted(cg, w, b.w);
                cb = add_weighted(cb, w, rc[u]);
                T = Tn;
                if ((__ballot(al != 0.f) & ~__ballot(stop)) != 0) {
                    if (lane == 0) Hl[nh] = (uint16_t)j;
                    ++nh;
                }
            }
            if (__ballot(!done) == 0) break;
        }
    }
    if (inside && !done) walk = end - beg;
    const float TF = T, PKr = cr, PKg = cg, PKb = cb;
    const float Qr = __fadd_rn(cr, __fmul_rn(TF, cfg.bg[0]));
    const float Qg = __fadd_rn(cg, __fmul_rn(TF, cfg.bg[1]));
    const float Qb = __fadd_rn(cb, __fmul_rn(TF, cfg.bg[2]));
    float er = 0.f, eg = 0.f, eb = 0.f;
    if (inside) {
        const int64_t pix = (int64_t)py * J.W + px;
        if (J.image) {
            J.image[3 * pix] = Qr;
            J.image[3 * pix + 1] = Qg;
            J.image[3 * pix + 2] = Qb;
        }
        if (se) {
            er = Qr - J.target[3 * pix];
            eg = Qg - J.target[3 * pix + 1];
            eb = Qb - J.target[3 * pix + 2];
        }
    }
    (void)PKr;
    (void)PKg;
    (void)PKb;
    if (n_out == 0) {
        __syncthreads();
        return;
    }

    // ---- removal sweep over the walked prefix
    if (threadIdx.x == 0) sm.misc[0] = 0;
    // per-entry sums start at zero (the flush clears what it reads)
    long long* const part64 = reinterpret_cast<long long*>(sm.part);   // FX: the sums as fixed point
    for (int j = threadIdx.x; j < n_out * B; j += NT) {
        if constexpr (FX) part64[j] = 0;
        else sm.part[j] = 0.f;
    }
    __syncthreads();
    if (walk > 0) atomicMax(&sm.misc[0], walk);
    __syncthreads();
    const int wmax = sm.misc[0];
    // this wave's longest walk bounds its entries; later ones contribute 0
    int wave_walk = walk;
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) wave_walk = max(wave_walk, __shfl_xor(wave_walk, m, 64));
    wave_walk = __builtin_amdgcn_readfirstlane(wave_walk);
    T = 1.f;
    float Rr = Qr, Rg = Qg, Rb = Qb;   // Q - P: colour still to come
    for (int base = 0; base < wmax; base += B) {
        const int cnt = min(B, wmax - base);
        // entries to revisit: those this wave blended when the batch is still the
        // one the blend sweep left in LDS, else those reaching the wave's rows
        const uint16_t* LL = Hl;
        int nv = nh;
        bool hits = true;
        if (staged != beg + base) {
            __syncthreads();
            stage<NT, TH>(J.proj, J.ids, beg + base, cnt, sm, qmax, tile_y0);
            staged = beg + base;
            __syncthreads();
            nl = __builtin_amdgcn_readfirstlane(
                wave_list<kRecWords>(reinterpret_cast<const uint32_t*>(sm.rec) + kRowsWord, cnt, row_lo, row_hi, L));
            nh = 0;
            LL = L;
            nv = nl;
            hits = false;
        }
        // entries of this wave's list from jlim on lie past every lane's walk
        const int jlim = __builtin_amdgcn_readfirstlane(min(cnt, wave_walk - base));
        nv = __builtin_amdgcn_readfirstlane(nv);
        for (int i = 0; i < nv; i += 4) {
            int js[4];
            list4(LL, i, js);
            if (js[0] >= jlim) break;
            // the group's valid slots (the list is increasing, so they are a prefix)
            int ng = 1;
#pragma unroll
            for (int u = 1; u < 4; ++u) ng += (ng == u && i + u < nv && js[u] < jlim) ? 1 : 0;
            float4 ra[4], rb[4];
            float rc[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int jj = u < ng ? js[u] : js[0];
                ra[u] = sm.rec[jj].a;
                rb[u] = sm.rec[jj].b;
                rc[u] = sm.rec[jj].c.x;
            }
            float l1v[4] = {0.f, 0.f, 0.f, 0.f}, imv[4] = {0.f, 0.f, 0.f, 0.f}, sev[4] = {0.f, 0.f, 0.f, 0.f};
            // branch-free: a slot past the group's valid prefix takes alpha = 0,
            // which leaves T and R unchanged and gives a zero removal effect
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int j = js[u];
                const float4 b = rb[u];
                const float al =
                    alpha_if(eval_gauss(ra[u], b, fx, fy), emin, amin, amax, u < ng && base + j < walk);
                const float w = __fmul_rn(T, al);
                const float c0 = b.z, c1 = b.w, c2 = rc[u];
                const float r0 = Rr, r1 = Rg, r2 = Rb;
                Rr = sub_weighted(Rr, w, c0);
                Rg = sub_weighted(Rg, w, c1);
                Rb = sub_weighted(Rb, w, c2);
                const float inv = inv_keep(al);
                const float dr = removal_delta(inv, Rr, r0);
                const float dg = removal_delta(inv, Rg, r1);
                const float db = removal_delta(inv, Rb, r2);
                l1v[u] = fabsf(dr) + fabsf(dg) + fabsf(db);
                if (SE) sev[u] = dr * dr + dg * dg + db * db + 2.f * (dr * er + dg * eg + db * eb);
                imv[u] = w;
                T = next_T(T, al);
            }
            // an entry of the blended list was blended by some lane, so only a
            // group of the full list can contribute nothing
            if (!hits && __ballot(imv[0] != 0.f || imv[1] != 0.f || imv[2] != 0.f || imv[3] != 0.f) == 0) continue;
            // lane u < 4 writes entry js[u] (only entries that are in the list)
            const int jw = lane == 0 ? js[0] : lane == 1 ? js[1] : lane == 2 ? js[2] : js[3];
            const bool writer = lane < ng;
            if (J.scores) {
                const float s = wave_sum4(l1v[0], l1v[1], l1v[2], l1v[3]);
                if (writer) {
                    if constexpr (FX) atomicAdd((unsigned long long*)&part64[o_l1 * B + jw], to_fixed(s));
                    else atomicAdd(&sm.part[o_l1 * B + jw], s);
                }
            }
            if (J.importance) {
                const float s = wave_sum4(imv[0], imv[1], imv[2], imv[3]);
                if (writer) {
                    if constexpr (FX) atomicAdd((unsigned long long*)&part64[o_im * B + jw], to_fixed(s));
                    else atomicAdd(&sm.part[o_im * B + jw], s);
                }
            }
            if (se) {
                const float s = wave_sum4(sev[0], sev[1], sev[2], sev[3]);
                if (writer) {
                    if constexpr (FX) atomicAdd((unsigned long long*)&part64[o_se * B + jw], to_fixed(s));
                    else atomicAdd(&sm.part[o_se * B + jw], s);
                }
            }
        }
        __syncthreads();
        for (int j = threadIdx.x; j < cnt; j += NT) {
            const uint32_t id = __float_as_uint(sm.rec[j].c.y);
            if constexpr (FX) {
                // the weight scales the exact sum (an int64 below 2^53 converts exactly), one rounding
                long long t[3] = {0, 0, 0};
#pragma unroll
                for (int o = 0; o < 3; ++o)
                    if (o < n_out) {
                        t[o] = part64[o * B + j];
                        part64[o * B + j] = 0;
                    }
                auto add = [&](float* out, long long v, float w) {
                    atomicAdd(reinterpret_cast<unsigned long long*>(out) + id,
                              (unsigned long long)__double2ll_rn((double)v * (double)w));
                };
                if (J.scores && t[o_l1] != 0) add(J.scores, t[o_l1], J.w_l1);
                if (J.importance && t[o_im] != 0) add(J.importance, t[o_im], J.w_im);
                if (se && t[o_se] != 0) add(J.scores_se, t[o_se], J.w_se);
            } else {
                float t[3] = {0.f, 0.f, 0.f};
#pragma unroll
                for (int o = 0; o < 3; ++o)
                    if (o < n_out) {
                        t[o] = sm.part[o * B + j];
                        sm.part[o * B + j] = 0.f;
                    }
                if (J.scores && t[o_l1] != 0.f) unsafeAtomicAdd(J.scores + id, t[o_l1] * J.w_l1);
                if (J.importance && t[o_im] != 0.f) unsafeAtomicAdd(J.importance + id, t[o_im] * J.w_im);
                if (se && t[o_se] != 0.f) unsafeAtomicAdd(J.scores_se + id, t[o_se] * J.w_se);
            }
        }
    }
    __syncthreads();
}

template <int TW, int TH>
__device__ inline Smem carve(char* base, int B) {
    constexpr int NW = (TW * TH + 63) / 64;
    Smem s;
    s.rec = reinterpret_cast<Rec*>(base);
    s.list = reinterpret_cast<uint16_t*>(s.rec + B);
    s.hits = s.list + NW * B;
    s.misc = reinterpret_cast<int*>(s.hits + NW * B);
    s.part = reinterpret_cast<float*>(s.misc + 4);
    return s;
}

template <int TW, int TH, bool SE, bool FX>
__global__ __launch_bounds__(TW * TH) __attribute__((amdgpu_waves_per_eu(7))) void k_render_score(ViewJobs jobs, potr_config cfg) {
    extern __shared__ __align__(16) char smem[];
    const Smem sm = carve<TW, TH>(smem, cfg.lds_batch);
    const ViewJob J = jobs.j[blockIdx.y];
    render_score_tile<TW, TH, SE, FX>(J, blockIdx.x, cfg, sm);
}

// Persistent form: items are (view job, tile) pairs numbered job-major;
// item_prefix[j] is the first item of job j (item_prefix[n_jobs] = total).
// waves per SIMD the persistent form is compiled for (its register budget)
constexpr int kPersistentWaves = 7;

template <int TW, int TH, bool SE, bool FX>
__global__ __launch_bounds__(TW * TH) __attribute__((amdgpu_waves_per_eu(kPersistentWaves))) void k_render_score_persistent(const ViewJob* __restrict__ jobs, int32_t n_jobs,
                                                                     const int64_t* __restrict__ item_prefix,
                                                                     int64_t* __restrict__ counter, potr_config cfg) {
    extern __shared__ __align__(16) char smem[];
    __shared__ int64_t s_item;   // the item this workgroup took (64-bit: totals may pass 2^31)
    const Smem sm = carve<TW, TH>(smem, cfg.lds_batch);
    const int64_t total = item_prefix[n_jobs];
    for (;;) {
        if (threadIdx.x == 0) s_item = (int64_t)atomicAdd((unsigned long long*)counter, 1ull);
        __syncthreads();
        const int64_t item = s_item;
        __syncthreads();
        if (item >= total) break;
        int lo = 0, hi = n_jobs - 1;      // last job with item_prefix[j] <= item
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (item_prefix[mid] <= item) lo = mid;
            else hi = mid - 1;
        }
        const ViewJob J = jobs[lo];
        render_score_tile<TW, TH, SE, FX>(J, (int)(item - item_prefix[lo]), cfg, sm);
    }
}

__global__ void k_zero_i64(int64_t* p) { *p = 0; }

__global__ void k_fixed_to_float(int64_t n, const long long* __restrict__ acc, float* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] = (float)((double)acc[i] * (1.0 / kFixedOne));
}

// per-entry sums: 4 bytes each, 8 in fixed point
template <int TW, int TH>
size_t smem_bytes(int B, int n_out, bool fx) {
    constexpr int NW = (TW * TH + 63) / 64;
    return (size_t)B * sizeof(Rec) + (size_t)NW * B * 4 + 16 + (size_t)n_out * B * (fx ? 8 : 4);
}

template <int TW, int TH, bool SE>
void launch_plain(const ViewJobs& jobs_dev, dim3 grid, size_t sm, const potr_config& cfg, bool fx, hipStream_t s) {
    if (fx) hipLaunchKernelGGL((k_render_score<TW, TH, SE, true>), grid, dim3(TW * TH), sm, s, jobs_dev, cfg);
    else hipLaunchKernelGGL((k_render_score<TW, TH, SE, false>), grid, dim3(TW * TH), sm, s, jobs_dev, cfg);
}

template <int TW, int TH, bool SE>
void launch_pers(const ViewJob* jobs_dev, int32_t n_jobs, const int64_t* item_prefix_dev, int64_t* counter_dev,
                 dim3 grid, size_t sm, const potr_config& cfg, bool fx, hipStream_t s) {
    if (fx)
        hipLaunchKernelGGL((k_render_score_persistent<TW, TH, SE, true>), grid, dim3(TW * TH), sm, s, jobs_dev,
                           n_jobs, item_prefix_dev, counter_dev, cfg);
    else
        hipLaunchKernelGGL((k_render_score_persistent<TW, TH, SE, false>), grid, dim3(TW * TH), sm, s, jobs_dev,
                           n_jobs, item_prefix_dev, counter_dev, cfg);
}

}  // namespace

size_t fused_smem_bytes(const potr_config& cfg, int n_out, bool fx) {
    if (cfg.tile_w == 8) return smem_bytes<8, 8>(cfg.lds_batch, n_out, fx);
    if (cfg.tile_w == 32) return smem_bytes<32, 8>(cfg.lds_batch, n_out, fx);
    return smem_bytes<16, 16>(cfg.lds_batch, n_out, fx);
}

potr_status launch_render_score(const ViewJobs& jobs_dev, int32_t n_views, int32_t tiles_per_view,
                                const potr_config& cfg, bool fx, hipStream_t s) {
    // the views of one call share their set of outputs
    const ViewJob& j0 = jobs_dev.j[0];
    const int n_out = (j0.scores ? 1 : 0) + (j0.importance ? 1 : 0) + (j0.scores_se ? 1 : 0);
    const size_t sm = fused_smem_bytes(cfg, n_out, fx);
    const dim3 grid(tiles_per_view, n_views);
    const bool se = jobs_dev.j[0].scores_se != nullptr;
    if (cfg.tile_w == 16 && cfg.tile_h == 16) {
        if (se) launch_plain<16, 16, true>(jobs_dev, grid, sm, cfg, fx, s);
        else launch_plain<16, 16, false>(jobs_dev, grid, sm, cfg, fx, s);
    } else if (cfg.tile_w == 8 && cfg.tile_h == 8) {
        if (se) launch_plain<8, 8, true>(jobs_dev, grid, sm, cfg, fx, s);
        else launch_plain<8, 8, false>(jobs_dev, grid, sm, cfg, fx, s);
    } else if (cfg.tile_w == 32 && cfg.tile_h == 8) {
        if (se) launch_plain<32, 8, true>(jobs_dev, grid, sm, cfg, fx, s);
        else launch_plain<32, 8, false>(jobs_dev, grid, sm, cfg, fx, s);
    } else {
        return fail(POTR_EUNSUPPORTED, "tile %dx%d not built", cfg.tile_w, cfg.tile_h);
    }
    return check_launch("k_render_score");
}

int persistent_grid(const potr_config& cfg, int n_out, bool fx) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess)
        cus = 256;
    const int threads = cfg.tile_w * cfg.tile_h;
    const size_t sm = fused_smem_bytes(cfg, n_out, fx);
    int by_waves = 4 * kPersistentWaves / ((threads + 63) / 64);   // 4 SIMDs per CU
    int by_lds = (int)((160 * 1024) / (sm + 256));
    int per_cu = by_waves < by_lds ? by_waves : by_lds;
    if (per_cu < 1) per_cu = 1;
    return cus * per_cu;
}

template <bool SE>
potr_status launch_persistent(const ViewJob* jobs_dev, int32_t n_jobs, const int64_t* item_prefix_dev,
                              int64_t* counter_dev, int32_t grid_size, const potr_config& cfg, int n_out, bool fx,
                              hipStream_t s) {
    const size_t sm = fused_smem_bytes(cfg, n_out, fx);
    const dim3 grid(grid_size);
    if (cfg.tile_w == 16 && cfg.tile_h == 16)
        launch_pers<16, 16, SE>(jobs_dev, n_jobs, item_prefix_dev, counter_dev, grid, sm, cfg, fx, s);
    else if (cfg.tile_w == 8 && cfg.tile_h == 8)
        launch_pers<8, 8, SE>(jobs_dev, n_jobs, item_prefix_dev, counter_dev, grid, sm, cfg, fx, s);
    else if (cfg.tile_w == 32 && cfg.tile_h == 8)
        launch_pers<32, 8, SE>(jobs_dev, n_jobs, item_prefix_dev, counter_dev, grid, sm, cfg, fx, s);
    else
        return fail(POTR_EUNSUPPORTED, "tile %dx%d not built", cfg.tile_w, cfg.tile_h);
    return check_launch("k_render_score_persistent");
}

potr_status launch_render_score_persistent(const ViewJob* jobs_dev, int32_t n_jobs, const int64_t* item_prefix_dev,
                                           int64_t* counter_dev, int32_t grid_size, const potr_config& cfg,
                                           bool with_se, int n_out, bool fx, hipStream_t s) {
    hipLaunchKernelGGL(k_zero_i64, dim3(1), dim3(1), 0, s, counter_dev);
    potr_status st = check_launch("k_zero_i64");
    if (st != POTR_OK) return st;
    return with_se ? launch_persistent<true>(jobs_dev, n_jobs, item_prefix_dev, counter_dev, grid_size, cfg, n_out,
                                             fx, s)
                   : launch_persistent<false>(jobs_dev, n_jobs, item_prefix_dev, counter_dev, grid_size, cfg, n_out,
                                              fx, s);
}

potr_status launch_fixed_to_float(int64_t n, const int64_t* acc, float* out, hipStream_t s) {
    if (n <= 0) return POTR_OK;
    const int blocks = (int)std::min<int64_t>(4096, (n + 255) / 256);
    hipLaunchKernelGGL(k_fixed_to_float, dim3(blocks), dim3(256), 0, s, n, (const long long*)acc, out);
    return check_launch("k_fixed_to_float");
}

}  // namespace potr
