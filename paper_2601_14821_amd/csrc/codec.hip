// The codec of the paper (Sec. 4.5): uniform attribute quantisation, octree
// geometry with the precision test, depth-first occupancy bytes, attributes in
// leaf order, zstd.
//
// Encoder, on the device: per splat the nearest camera eye and its precision
// bound, its cell on a 2^D grid and the Morton code of that cell (3 bits per
// level, octant c = x | y << 1 | z << 2, the root's digit on top); a radix sort
// of the codes (ties keep index order) puts the splats in the depth-first leaf
// order of the octree. A splat's leaf depth follows from its sorted neighbours:
// every node down to one level below the longer common prefix with either
// neighbour holds another splat and splits; from there its node holds it alone
// and splits until the precision test passes (or the depth cap is reached).
// The attributes are quantised straight into leaf order. The occupancy bytes
// follow from the same order: splat k enters the tree one level below its
// common prefix with splat k-1, appends the bytes of its new nodes (one child
// each, as far as it knows) and of its leaf at a scanned offset, and sets its
// octant bit in the byte of the node where it branches off (found, per depth,
// by a running maximum over the splats that entered at or above it). zstd runs
// on the host.
//
// Decoder, on the host: zstd, then a depth-first walk of the bytes that gives
// the leaf centres in the same order as the attribute streams, which are
// dequantised in place.
//
// Every FP64 step is an IEEE operation in the order of the reading the oracle
// states (no contraction), so the bitstream is the same byte for byte.
#include <dlfcn.h>

#include <cmath>
#include <cstring>
#include <mutex>
#include <vector>

#include <hipcub/hipcub.hpp>

#include "common.h"

namespace potr {
namespace {

constexpr uint32_t kMagic = 0x52544F50u;   // "POTR"
constexpr uint32_t kVersion = 1;
constexpr int kThreads = 256;
constexpr int kBoundBlocks = 512;

#pragma pack(push, 1)
struct Header {
    uint32_t magic, version;
    uint64_t n;
    uint32_t depth, sh_degree;
    double lo[3], size;
    double sf[4];   // scale, rotation, opacity, SH
    uint64_t n_nodes, n_caps;
};
#pragma pack(pop)
static_assert(sizeof(Header) == 104, "header layout");

int n_streams(int deg) { return 7 + 3 * (deg + 1) * (deg + 1); }

// ---------------------------------------------------------------- device

// Per-block minimum and maximum of the positions per axis: part[b][0..2] the
// minima, part[b][3..5] the maxima.
__global__ __launch_bounds__(kThreads) void k_codec_bounds(int64_t N, const float* __restrict__ means,
                                                          float* __restrict__ part) {
    __shared__ float s[6][kThreads];
    float lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x; i < N; i += (int64_t)gridDim.x * kThreads) {
#pragma unroll
        for (int a = 0; a < 3; ++a) {
            const float v = means[3 * i + a];
            lo[a] = fminf(lo[a], v);
            hi[a] = fmaxf(hi[a], v);
        }
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        s[a][threadIdx.x] = lo[a];
        s[3 + a][threadIdx.x] = hi[a];
    }
    __syncthreads();
    for (int h = kThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                s[a][threadIdx.x] = fminf(s[a][threadIdx.x], s[a][threadIdx.x + h]);
                s[3 + a][threadIdx.x] = fmaxf(s[3 + a][threadIdx.x], s[3 + a][threadIdx.x + h]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[6 * blockIdx.x + threadIdx.x] = s[threadIdx.x][0];
}

struct Grid {
    double lo[3];
    double size;
    double scale;   // 2^D / size
    int depth;
};

__device__ inline uint32_t grid_cell(double v, double lo, double scale, int D) {
#pragma clang fp contract(off)
    const double c = floor((v - lo) * scale);
    const double top = (double)((1u << D) - 1u);
    return (uint32_t)(c < 0.0 ? 0.0 : (c > top ? top : c));
}

// Per splat: the smallest squared distance to a camera eye, the precision
// bound max(gamma^2, beta^2 d2min), and the Morton code of its grid cell.
__global__ __launch_bounds__(kThreads) void k_codec_prep(int64_t N, const float* __restrict__ means,
                                                        const double* __restrict__ eyes, int n_eyes, Grid G,
                                                        double gamma2, double beta2, double* __restrict__ thr2,
                                                        uint64_t* __restrict__ code, uint32_t* __restrict__ idx) {
#pragma clang fp contract(off)
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= N) return;
    const double m0 = means[3 * i], m1 = means[3 * i + 1], m2 = means[3 * i + 2];
    double best = INFINITY;
    for (int e = 0; e < n_eyes; ++e) {
        const double d0 = m0 - eyes[3 * e], d1 = m1 - eyes[3 * e + 1], d2 = m2 - eyes[3 * e + 2];
        const double q = (d0 * d0 + d1 * d1) + d2 * d2;
        best = q < best ? q : best;
    }
    const double b = beta2 * best;
    thr2[i] = gamma2 > b ? gamma2 : b;
    const uint32_t X = grid_cell(m0, G.lo[0], G.scale, G.depth);
    const uint32_t Y = grid_cell(m1, G.lo[1], G.scale, G.depth);
    const uint32_t Z = grid_cell(m2, G.lo[2], G.scale, G.depth);
    uint64_t c = 0;
    for (int l = G.depth - 1; l >= 0; --l)
        c = (c << 3) | (uint64_t)(((X >> l) & 1u) | (((Y >> l) & 1u) << 1) | (((Z >> l) & 1u) << 2));
    code[i] = c;
    idx[i] = (uint32_t)i;
}

// Levels two Morton codes of D levels share from the root (D when equal).
__device__ inline int common_levels(uint64_t a, uint64_t b, int D) {
    const uint64_t x = a ^ b;
    if (x == 0) return D;
    const int h = 63 - __clzll((long long)x);   // highest differing bit
    return D - 1 - h / 3;
}

// Per sorted splat: the depth where it enters the tree (one below its common
// prefix with the previous splat; D + 1 when it shares the previous splat's
// cap leaf) and its leaf depth.
__global__ __launch_bounds__(kThreads) void k_codec_leaf(int64_t N, const uint64_t* __restrict__ code,
                                                        const uint32_t* __restrict__ idx,
                                                        const float* __restrict__ means,
                                                        const double* __restrict__ thr2, Grid G,
                                                        uint8_t* __restrict__ enter, uint8_t* __restrict__ leaf) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    const int D = G.depth;
    const uint64_t c = code[k];
    const int lp = k > 0 ? common_levels(code[k - 1], c, D) : -1;
    const int ln = k + 1 < N ? common_levels(c, code[k + 1], D) : -1;
    const int sep = (lp > ln ? lp : ln) + 1;   // first depth where the node holds this splat alone
    int depth = D;
    if (sep < D) {
        const uint32_t i = idx[k];
        const double m[3] = {means[3 * i], means[3 * i + 1], means[3 * i + 2]};
        const double t2 = thr2[i];
        uint32_t cell[3] = {0u, 0u, 0u};
        for (int l = D - 1; l >= 0; --l) {
            const uint32_t dg = (uint32_t)(c >> (3 * l)) & 7u;
            cell[0] = (cell[0] << 1) | (dg & 1u);
            cell[1] = (cell[1] << 1) | ((dg >> 1) & 1u);
            cell[2] = (cell[2] << 1) | ((dg >> 2) & 1u);
        }
        for (int L = sep; L < D; ++L) {
            const double step = G.size * ldexp(1.0, -L);
            double dd[3];
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const double ctr = G.lo[a] + ((double)(cell[a] >> (D - L)) + 0.5) * step;
                dd[a] = m[a] - ctr;
            }
            const double q = (dd[0] * dd[0] + dd[1] * dd[1]) + dd[2] * dd[2];
            if (q < t2) {
                depth = L;
                break;
            }
        }
    }
    enter[k] = (uint8_t)(lp + 1);
    leaf[k] = (uint8_t)depth;
}

struct Quant {
    double sf_scale, sf_rot, sf_opac, sf_sh;
    int nsh;
};

// floor(1/2 + x SF) as int64; sets *bad when it leaves the int32 range.
__device__ inline int64_t quant(double x, double sf, bool& bad) {
#pragma clang fp contract(off)
    const double v = floor(0.5 + x * sf);
    if (!(v >= -2147483648.0 && v <= 2147483647.0)) {
        bad = true;
        return 0;
    }
    return (int64_t)v;
}

// Every attribute of sorted splat k, quantised into its stream at column k:
// opacity; scale x, y, z; the unit quaternion's x, y, z (w >= 0); SH
// coefficient j channel r, g, b (j = 0 as the difference to splat k - 1).
__global__ __launch_bounds__(kThreads) void k_codec_attr(int64_t N, const uint32_t* __restrict__ idx,
                                                        const float* __restrict__ scales,
                                                        const float* __restrict__ quats,
                                                        const float* __restrict__ opac, const float* __restrict__ sh,
                                                        Quant Q, int32_t* __restrict__ st, int* __restrict__ flag) {
#pragma clang fp contract(off)
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    const uint32_t i = idx[k];
    bool bad = false;
    int64_t v[7];
    v[0] = quant(opac[i], Q.sf_opac, bad);
#pragma unroll
    for (int a = 0; a < 3; ++a) v[1 + a] = quant(scales[3 * i + a], Q.sf_scale, bad);
    const double q0 = quats[4 * i], q1 = quats[4 * i + 1], q2 = quats[4 * i + 2], q3 = quats[4 * i + 3];
    const double n2 = ((q0 * q0 + q1 * q1) + q2 * q2) + q3 * q3;
    double u[4] = {1.0, 0.0, 0.0, 0.0};
    if (n2 != 0.0) {
        const double nrm = sqrt(n2);
        u[0] = q0 / nrm;
        u[1] = q1 / nrm;
        u[2] = q2 / nrm;
        u[3] = q3 / nrm;
    }
    if (u[0] < 0.0) {
#pragma unroll
        for (int a = 0; a < 4; ++a) u[a] = -u[a];
    }
#pragma unroll
    for (int a = 0; a < 3; ++a) v[4 + a] = quant(u[1 + a], Q.sf_rot, bad);
#pragma unroll
    for (int s = 0; s < 7; ++s) st[(int64_t)s * N + k] = (int32_t)v[s];
    const float* c = sh + 48 * (int64_t)i;
    const float* cp = k > 0 ? sh + 48 * (int64_t)idx[k - 1] : nullptr;
    for (int j = 0; j < Q.nsh; ++j) {
#pragma unroll
        for (int ch = 0; ch < 3; ++ch) {
            int64_t q = quant(c[3 * j + ch], Q.sf_sh, bad);
            if (j == 0 && cp) {
                q -= quant(cp[ch], Q.sf_sh, bad);
                if (q < -2147483648LL || q > 2147483647LL) bad = true;
            }
            st[(int64_t)(7 + 3 * j + ch) * N + k] = (int32_t)q;
        }
    }
    if (bad) atomicOr(flag, 1);
}

// The octree bytes, depth first (as the recursion would write them). A sorted
// splat appends the bytes of its new nodes, from the depth where it enters the
// tree to its leaf (none when it shares the previous splat's cap leaf): each of
// its internal nodes starts with the bit of its own child, its leaf is 0. The
// node where splat k branches off (at depth enter[k] - 1) was appended by the
// last splat before k that entered the tree at or above that depth; k sets its
// octant bit there.
__device__ inline uint32_t digit_at(uint64_t c, int level, int D) {   // level 1..D
    return (uint32_t)(c >> (3 * (D - level))) & 7u;
}

__global__ __launch_bounds__(kThreads) void k_codec_count(int64_t N, const uint8_t* __restrict__ enter,
                                                         const uint8_t* __restrict__ leaf, int D,
                                                         uint64_t* __restrict__ nb, uint32_t* __restrict__ capf) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    const int e = enter[k], d = leaf[k];
    nb[k] = e <= D ? (uint64_t)(d - e + 1) : 0ull;
    capf[k] = (e <= D && d == D) ? 1u : 0u;
}

__global__ __launch_bounds__(kThreads) void k_codec_own(int64_t N, const uint64_t* __restrict__ code,
                                                       const uint8_t* __restrict__ enter,
                                                       const uint8_t* __restrict__ leaf,
                                                       const uint64_t* __restrict__ off, int D,
                                                       uint8_t* __restrict__ nodes) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    const int e = enter[k], d = leaf[k];
    if (e > D) return;
    const uint64_t c = code[k], p = off[k];
    for (int L = e; L < d; ++L) nodes[p + (uint64_t)(L - e)] = (uint8_t)(1u << digit_at(c, L + 1, D));
    nodes[p + (uint64_t)(d - e)] = 0;
}

// f[k] = k where splat k entered the tree at depth <= l, else -1 (the running
// maximum of f is then the last such splat at or before each position)
__global__ __launch_bounds__(kThreads) void k_codec_flag(int64_t N, const uint8_t* __restrict__ enter, int l,
                                                        int32_t* __restrict__ f) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    f[k] = (int)enter[k] <= l ? (int32_t)k : -1;
}

__global__ __launch_bounds__(kThreads) void k_codec_branch(int64_t N, const uint64_t* __restrict__ code,
                                                          const uint8_t* __restrict__ enter,
                                                          const uint64_t* __restrict__ off,
                                                          const int32_t* __restrict__ last, int l, int D,
                                                          uint32_t* __restrict__ words) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N) return;
    const int e = enter[k];
    if (e != l + 1 || e > D) return;   // branches off at depth l (k > 0 here: splat 0 enters at 0)
    const int32_t a = last[k - 1];      // >= 0: splat 0 entered at depth 0
    const uint64_t pos = off[a] + (uint64_t)(l - (int)enter[a]);
    atomicOr(words + (pos >> 2), (1u << digit_at(code[k], l + 1, D)) << (8 * (uint32_t)(pos & 3)));
}

// The splat count of each leaf at the depth cap: the splat that opens it and
// the duplicates right behind it.
__global__ __launch_bounds__(kThreads) void k_codec_caps(int64_t N, const uint8_t* __restrict__ enter,
                                                        const uint32_t* __restrict__ capf,
                                                        const uint32_t* __restrict__ capoff, int D,
                                                        uint32_t* __restrict__ caps) {
    const int64_t k = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (k >= N || !capf[k]) return;
    int64_t j = k + 1;
    while (j < N && (int)enter[j] > D) ++j;
    caps[capoff[k]] = (uint32_t)(j - k);
}

// ---------------------------------------------------------------- host

struct EncWs {
    double* eyes;
    float* part;
    double* thr2;
    uint64_t* code_in;
    uint64_t* code;
    uint32_t* idx_in;
    uint32_t* idx;
    uint8_t* enter;
    uint8_t* leaf;
    int32_t* streams;
    int* flag;
    uint64_t* nb;       // bytes per sorted splat (in the codes' first buffer, free after the sort)
    uint64_t* off;      // their exclusive scan (in the precision bounds' buffer, free after the leaves)
    uint32_t* capf;
    uint32_t* capoff;
    int32_t* f;
    int32_t* last;
    uint8_t* nodes;     // N * (21 + 1) bytes at most, rounded to words
    uint32_t* caps;
    uint64_t* totals;   // n_nodes, n_caps
    void* sort_tmp;
    size_t sort_bytes;
    size_t bytes;
};

// scratch of the library's radix sort and scans (size queries only: they read
// no memory and cannot fail for valid sizes)
size_t sort_tmp_bytes(int64_t N) {
    const int n = (int)std::max<int64_t>(N, 1);
    size_t a = 0, b = 0, c = 0, d = 0;
    (void)hipcub::DeviceRadixSort::SortPairs(nullptr, a, (const uint64_t*)nullptr, (uint64_t*)nullptr,
                                             (const uint32_t*)nullptr, (uint32_t*)nullptr, n, 0, 64);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, b, (const uint64_t*)nullptr, (uint64_t*)nullptr, n);
    (void)hipcub::DeviceScan::ExclusiveSum(nullptr, c, (const uint32_t*)nullptr, (uint32_t*)nullptr, n);
    (void)hipcub::DeviceScan::InclusiveScan(nullptr, d, (const int32_t*)nullptr, (int32_t*)nullptr, hipcub::Max(), n);
    return std::max(std::max(a, b), std::max(c, d));
}

EncWs enc_layout(int64_t N, int deg, int n_cams, char* base) {
    EncWs w{};
    size_t off = 0;
    auto take = [&](size_t n) {
        const size_t o = off;
        off += align_up(n > 0 ? n : 1);
        return base ? base + o : nullptr;
    };
    const size_t n = (size_t)std::max<int64_t>(N, 1);
    w.eyes = (double*)take((size_t)n_cams * 3 * 8);
    w.part = (float*)take((size_t)kBoundBlocks * 6 * 4);
    w.thr2 = (double*)take(n * 8);
    w.code_in = (uint64_t*)take(n * 8);
    w.code = (uint64_t*)take(n * 8);
    w.idx_in = (uint32_t*)take(n * 4);
    w.idx = (uint32_t*)take(n * 4);
    w.enter = (uint8_t*)take(n);
    w.leaf = (uint8_t*)take(n);
    w.streams = (int32_t*)take(n * (size_t)n_streams(deg) * 4);
    w.flag = (int*)take(4);
    w.nb = w.code_in;
    w.off = (uint64_t*)w.thr2;
    w.capf = (uint32_t*)take(n * 4);
    w.capoff = (uint32_t*)take(n * 4);
    w.f = (int32_t*)take(n * 4);
    w.last = (int32_t*)take(n * 4);
    w.nodes = (uint8_t*)take(align_up(n * 22, 4));
    w.caps = (uint32_t*)take(n * 4);
    w.totals = (uint64_t*)take(16);
    w.sort_bytes = sort_tmp_bytes(N);
    w.sort_tmp = take(w.sort_bytes);
    w.bytes = off;
    return w;
}

potr_status hip_ok(hipError_t e, const char* what) {
    if (e != hipSuccess) return fail(POTR_EHIP, "%s: %s", what, hipGetErrorString(e));
    return POTR_OK;
}

bool finite_pos(double x) { return x > 0.0 && x < 1e300; }

// ---- zstd (the system's libzstd, loaded on first use)
struct Zstd {
    size_t (*bound)(size_t) = nullptr;
    size_t (*compress)(void*, size_t, const void*, size_t, int) = nullptr;
    size_t (*decompress)(void*, size_t, const void*, size_t) = nullptr;
    unsigned (*is_error)(size_t) = nullptr;
    unsigned long long (*content_size)(const void*, size_t) = nullptr;
    bool ok = false;
};

const Zstd& zstd() {
    static Zstd z;
    static std::once_flag once;
    std::call_once(once, [] {
        void* h = dlopen("libzstd.so.1", RTLD_NOW | RTLD_LOCAL);
        if (!h) return;
        z.bound = (size_t(*)(size_t))dlsym(h, "ZSTD_compressBound");
        z.compress = (size_t(*)(void*, size_t, const void*, size_t, int))dlsym(h, "ZSTD_compress");
        z.decompress = (size_t(*)(void*, size_t, const void*, size_t))dlsym(h, "ZSTD_decompress");
        z.is_error = (unsigned (*)(size_t))dlsym(h, "ZSTD_isError");
        z.content_size = (unsigned long long (*)(const void*, size_t))dlsym(h, "ZSTD_getFrameContentSize");
        z.ok = z.bound && z.compress && z.decompress && z.is_error && z.content_size;
    });
    return z;
}

bool read_header(const uint8_t* raw, size_t raw_bytes, Header& h) {
    if (!raw || raw_bytes < sizeof(Header)) return false;
    std::memcpy(&h, raw, sizeof(Header));
    if (h.magic != kMagic || h.version != kVersion || h.depth < 1 || h.depth > 21 || h.sh_degree > 3) return false;
    if (h.n >= (uint64_t(1) << 31) || h.n_nodes > h.n * (h.depth + 1) || h.n_caps > h.n) return false;
    const uint64_t need = sizeof(Header) + h.n_nodes + 4 * h.n_caps + 4 * h.n * (uint64_t)n_streams((int)h.sh_degree);
    return need == raw_bytes;
}

}  // namespace
}  // namespace potr

using namespace potr;

extern "C" {

potr_status potr_codec_workspace_size(int64_t N, int32_t sh_degree, int32_t n_cams, size_t* bytes) {
    if (!bytes || N < 0 || N >= (int64_t(1) << 31) || sh_degree < 0 || sh_degree > 3 || n_cams < 1)
        return fail(POTR_EINVAL, "bad argument");
    *bytes = enc_layout(N, sh_degree, n_cams, nullptr).bytes;
    return POTR_OK;
}

potr_status potr_codec_max_bytes(int64_t N, int32_t sh_degree, int32_t max_depth, size_t* bytes) {
    if (!bytes || N < 0 || N >= (int64_t(1) << 31) || sh_degree < 0 || sh_degree > 3 || max_depth < 1 ||
        max_depth > 21)
        return fail(POTR_EINVAL, "bad argument");
    *bytes = sizeof(Header) + (size_t)N * (max_depth + 1) + 4 * (size_t)N + 4 * (size_t)N * n_streams(sh_degree);
    return POTR_OK;
}

potr_status potr_codec_encode(int64_t N, const float* means, const float* scales, const float* quats,
                              const float* opacities, const float* sh, int32_t sh_degree, const potr_camera* cams,
                              int32_t n_cams, const potr_codec_params* prm, void* ws, size_t ws_bytes, uint8_t* raw,
                              size_t raw_cap, size_t* raw_bytes, uint32_t* leaf_order, void* stream) {
    if (N < 0 || N >= (int64_t(1) << 31)) return fail(POTR_EINVAL, "N = %lld", (long long)N);
    if (sh_degree < 0 || sh_degree > 3) return fail(POTR_EINVAL, "sh_degree %d not in 0..3", sh_degree);
    if (!prm || !cams || n_cams < 1 || !raw_bytes || !raw) return fail(POTR_EINVAL, "NULL argument");
    if (N > 0 && (!means || !scales || !quats || !opacities || !sh || !ws)) return fail(POTR_EINVAL, "NULL buffer");
    const int D = prm->max_depth;
    if (D < 1 || D > 21) return fail(POTR_EINVAL, "max_depth %d not in 1..21", D);
    if (!finite_pos(prm->sf_scale) || !finite_pos(prm->sf_rot) || !finite_pos(prm->sf_opac) ||
        !finite_pos(prm->sf_sh))
        return fail(POTR_EINVAL, "scale factors must be positive and finite");
    if (!(prm->beta >= 0.0) || prm->beta > 1e150 || !(prm->gamma >= 0.0) || prm->gamma > 1e150)
        return fail(POTR_EINVAL, "beta and gamma must be non-negative and finite");
    const EncWs w = enc_layout(N, sh_degree, n_cams, (char*)ws);
    if (N > 0 && ws_bytes < w.bytes) return fail(POTR_ECAPACITY, "codec workspace %zu < %zu bytes", ws_bytes, w.bytes);
    hipStream_t s = (hipStream_t)stream;
    const int S = n_streams(sh_degree);

    Header h{};
    h.magic = kMagic;
    h.version = kVersion;
    h.n = (uint64_t)N;
    h.depth = (uint32_t)D;
    h.sh_degree = (uint32_t)sh_degree;
    h.size = 1.0;
    h.sf[0] = prm->sf_scale;
    h.sf[1] = prm->sf_rot;
    h.sf[2] = prm->sf_opac;
    h.sf[3] = prm->sf_sh;
    uint64_t n_nodes = 0, n_caps = 0;
    potr_status st = POTR_OK;
    if (N > 0) {
        // root cube
        const int nb = (int)std::min<int64_t>(kBoundBlocks, ceil_div(N, kThreads));
        hipLaunchKernelGGL(k_codec_bounds, dim3(nb), dim3(kThreads), 0, s, N, means, w.part);
        if ((st = check_launch("k_codec_bounds")) != POTR_OK) return st;
        std::vector<float> part((size_t)nb * 6);
        if ((st = hip_ok(hipMemcpyAsync(part.data(), w.part, part.size() * 4, hipMemcpyDeviceToHost, s), "bounds")))
            return st;
        if ((st = hip_ok(hipStreamSynchronize(s), "bounds"))) return st;
        float lo[3], hi[3];
        for (int a = 0; a < 3; ++a) {
            lo[a] = part[a];
            hi[a] = part[3 + a];
            for (int b = 1; b < nb; ++b) {
                lo[a] = std::fmin(lo[a], part[6 * b + a]);
                hi[a] = std::fmax(hi[a], part[6 * b + 3 + a]);
            }
        }
        if (!(std::isfinite(lo[0]) && std::isfinite(lo[1]) && std::isfinite(lo[2]) && std::isfinite(hi[0]) &&
              std::isfinite(hi[1]) && std::isfinite(hi[2])))
            return fail(POTR_EINVAL, "positions must be finite");
        double ext = 0.0;
        for (int a = 0; a < 3; ++a) {
            h.lo[a] = (double)lo[a];
            const double e = (double)hi[a] - h.lo[a];
            ext = e > ext ? e : ext;
        }
        h.size = ext > 0.0 ? ext * (1.0 + std::ldexp(1.0, -20)) : 1.0;
        Grid G{};
        for (int a = 0; a < 3; ++a) G.lo[a] = h.lo[a];
        G.size = h.size;
        G.scale = std::ldexp(1.0, D) / h.size;
        G.depth = D;
        // camera eyes, -R^T t
        std::vector<double> eyes((size_t)n_cams * 3);
        for (int c = 0; c < n_cams; ++c) {
            const potr_camera& cm = cams[c];
            for (int k = 0; k < 3; ++k) {
                const double s0 = (double)cm.R[k] * (double)cm.t[0];
                const double s1 = (double)cm.R[3 + k] * (double)cm.t[1];
                const double s2 = (double)cm.R[6 + k] * (double)cm.t[2];
                eyes[3 * c + k] = -((s0 + s1) + s2);
            }
        }
        if ((st = hip_ok(hipMemcpyAsync(w.eyes, eyes.data(), eyes.size() * 8, hipMemcpyHostToDevice, s), "eyes")))
            return st;
        const dim3 grid((unsigned)ceil_div(N, kThreads));
        hipLaunchKernelGGL(k_codec_prep, grid, dim3(kThreads), 0, s, N, means, (const double*)w.eyes, n_cams, G,
                           prm->gamma * prm->gamma, prm->beta * prm->beta, w.thr2, w.code_in, w.idx_in);
        if ((st = check_launch("k_codec_prep")) != POTR_OK) return st;
        size_t tb = w.sort_bytes;
        if ((st = hip_ok(hipcub::DeviceRadixSort::SortPairs(w.sort_tmp, tb, (const uint64_t*)w.code_in, w.code,
                                                             (const uint32_t*)w.idx_in, w.idx, (int)N, 0, 3 * D, s),
                         "radix sort of the Morton codes")))
            return st;
        hipLaunchKernelGGL(k_codec_leaf, grid, dim3(kThreads), 0, s, N, (const uint64_t*)w.code,
                           (const uint32_t*)w.idx, means, (const double*)w.thr2, G, w.enter, w.leaf);
        if ((st = check_launch("k_codec_leaf")) != POTR_OK) return st;
        if ((st = hip_ok(hipMemsetAsync(w.flag, 0, 4, s), "clear flag"))) return st;
        const Quant Q{prm->sf_scale, prm->sf_rot, prm->sf_opac, prm->sf_sh, (sh_degree + 1) * (sh_degree + 1)};
        hipLaunchKernelGGL(k_codec_attr, grid, dim3(kThreads), 0, s, N, (const uint32_t*)w.idx, scales, quats,
                           opacities, sh, Q, w.streams, w.flag);
        if ((st = check_launch("k_codec_attr")) != POTR_OK) return st;
        if (leaf_order &&
            (st = hip_ok(hipMemcpyAsync(leaf_order, w.idx, (size_t)N * 4, hipMemcpyDeviceToDevice, s), "leaf order")))
            return st;
        // the octree bytes and the cap-leaf counts, on the device
        hipLaunchKernelGGL(k_codec_count, grid, dim3(kThreads), 0, s, N, (const uint8_t*)w.enter,
                           (const uint8_t*)w.leaf, D, w.nb, w.capf);
        if ((st = check_launch("k_codec_count")) != POTR_OK) return st;
        tb = w.sort_bytes;
        if ((st = hip_ok(hipcub::DeviceScan::ExclusiveSum(w.sort_tmp, tb, (const uint64_t*)w.nb, w.off, (int)N, s),
                         "scan of the node bytes")))
            return st;
        tb = w.sort_bytes;
        if ((st = hip_ok(hipcub::DeviceScan::ExclusiveSum(w.sort_tmp, tb, (const uint32_t*)w.capf, w.capoff, (int)N, s),
                         "scan of the cap leaves")))
            return st;
        hipLaunchKernelGGL(k_codec_own, grid, dim3(kThreads), 0, s, N, (const uint64_t*)w.code,
                           (const uint8_t*)w.enter, (const uint8_t*)w.leaf, (const uint64_t*)w.off, D, w.nodes);
        if ((st = check_launch("k_codec_own")) != POTR_OK) return st;
        for (int l = 0; l < D; ++l) {
            hipLaunchKernelGGL(k_codec_flag, grid, dim3(kThreads), 0, s, N, (const uint8_t*)w.enter, l, w.f);
            if ((st = check_launch("k_codec_flag")) != POTR_OK) return st;
            tb = w.sort_bytes;
            if ((st = hip_ok(hipcub::DeviceScan::InclusiveScan(w.sort_tmp, tb, (const int32_t*)w.f, w.last,
                                                                hipcub::Max(), (int)N, s),
                             "running last entry")))
                return st;
            hipLaunchKernelGGL(k_codec_branch, grid, dim3(kThreads), 0, s, N, (const uint64_t*)w.code,
                               (const uint8_t*)w.enter, (const uint64_t*)w.off, (const int32_t*)w.last, l, D,
                               (uint32_t*)w.nodes);
            if ((st = check_launch("k_codec_branch")) != POTR_OK) return st;
        }
        hipLaunchKernelGGL(k_codec_caps, grid, dim3(kThreads), 0, s, N, (const uint8_t*)w.enter,
                           (const uint32_t*)w.capf, (const uint32_t*)w.capoff, D, w.caps);
        if ((st = check_launch("k_codec_caps")) != POTR_OK) return st;
        uint64_t last_off = 0, last_nb = 0;
        uint32_t last_capoff = 0, last_capf = 0;
        int flag = 0;
        if ((st = hip_ok(hipMemcpyAsync(&last_off, w.off + (N - 1), 8, hipMemcpyDeviceToHost, s), "totals")) ||
            (st = hip_ok(hipMemcpyAsync(&last_nb, w.nb + (N - 1), 8, hipMemcpyDeviceToHost, s), "totals")) ||
            (st = hip_ok(hipMemcpyAsync(&last_capoff, w.capoff + (N - 1), 4, hipMemcpyDeviceToHost, s), "totals")) ||
            (st = hip_ok(hipMemcpyAsync(&last_capf, w.capf + (N - 1), 4, hipMemcpyDeviceToHost, s), "totals")) ||
            (st = hip_ok(hipMemcpyAsync(&flag, w.flag, 4, hipMemcpyDeviceToHost, s), "flag")) ||
            (st = hip_ok(hipStreamSynchronize(s), "codec")))
            return st;
        if (flag) return fail(POTR_EINVAL, "a quantised value leaves the int32 range");
        n_nodes = last_off + last_nb;
        n_caps = (uint64_t)last_capoff + last_capf;
    }
    h.n_nodes = n_nodes;
    h.n_caps = n_caps;
    const size_t total = sizeof(Header) + (size_t)n_nodes + 4 * (size_t)n_caps + 4 * (size_t)N * S;
    *raw_bytes = total;
    if (total > raw_cap) return fail(POTR_ECAPACITY, "bitstream of %zu bytes, buffer of %zu", total, raw_cap);
    uint8_t* p = raw;
    std::memcpy(p, &h, sizeof(Header));
    p += sizeof(Header);
    if (n_nodes > 0 &&
        (st = hip_ok(hipMemcpyAsync(p, w.nodes, (size_t)n_nodes, hipMemcpyDeviceToHost, s), "node bytes")))
        return st;
    p += n_nodes;
    if (n_caps > 0 && (st = hip_ok(hipMemcpyAsync(p, w.caps, 4 * (size_t)n_caps, hipMemcpyDeviceToHost, s), "caps")))
        return st;
    p += 4 * n_caps;
    if (N > 0) {
        if ((st = hip_ok(hipMemcpyAsync(p, w.streams, 4 * (size_t)N * S, hipMemcpyDeviceToHost, s), "streams")))
            return st;
        if ((st = hip_ok(hipStreamSynchronize(s), "streams"))) return st;
    }
    return POTR_OK;
}

potr_status potr_codec_compress_bound(size_t raw_bytes, size_t* bytes) {
    const Zstd& z = zstd();
    if (!z.ok) return fail(POTR_EUNSUPPORTED, "libzstd.so.1 not found");
    if (!bytes) return fail(POTR_EINVAL, "NULL argument");
    *bytes = z.bound(raw_bytes);
    return POTR_OK;
}

potr_status potr_codec_compress(const uint8_t* raw, size_t raw_bytes, int32_t level, uint8_t* out, size_t out_cap,
                                size_t* out_bytes) {
    const Zstd& z = zstd();
    if (!z.ok) return fail(POTR_EUNSUPPORTED, "libzstd.so.1 not found");
    if (!raw || !out || !out_bytes) return fail(POTR_EINVAL, "NULL argument");
    const size_t n = z.compress(out, out_cap, raw, raw_bytes, level);
    if (z.is_error(n)) return fail(POTR_ECAPACITY, "zstd compression failed (buffer of %zu bytes)", out_cap);
    *out_bytes = n;
    return POTR_OK;
}

potr_status potr_codec_decompressed_size(const uint8_t* comp, size_t comp_bytes, size_t* raw_bytes) {
    const Zstd& z = zstd();
    if (!z.ok) return fail(POTR_EUNSUPPORTED, "libzstd.so.1 not found");
    if (!comp || !raw_bytes) return fail(POTR_EINVAL, "NULL argument");
    const unsigned long long n = z.content_size(comp, comp_bytes);
    if (n >= (1ull << 62)) return fail(POTR_EINVAL, "not a zstd frame with a content size");
    *raw_bytes = (size_t)n;
    return POTR_OK;
}

potr_status potr_codec_decompress(const uint8_t* comp, size_t comp_bytes, uint8_t* raw, size_t raw_cap,
                                  size_t* raw_bytes) {
    size_t need = 0;
    potr_status st = potr_codec_decompressed_size(comp, comp_bytes, &need);
    if (st != POTR_OK) return st;
    if (!raw || !raw_bytes) return fail(POTR_EINVAL, "NULL argument");
    *raw_bytes = need;
    if (need > raw_cap) return fail(POTR_ECAPACITY, "bitstream of %zu bytes, buffer of %zu", need, raw_cap);
    const Zstd& z = zstd();
    const size_t n = z.decompress(raw, raw_cap, comp, comp_bytes);
    if (z.is_error(n) || n != need) return fail(POTR_EINVAL, "zstd decompression failed");
    return POTR_OK;
}

potr_status potr_codec_info(const uint8_t* raw, size_t raw_bytes, int64_t* N, int32_t* sh_degree) {
    Header h;
    if (!read_header(raw, raw_bytes, h)) return fail(POTR_EINVAL, "not a bitstream of this codec");
    if (N) *N = (int64_t)h.n;
    if (sh_degree) *sh_degree = (int32_t)h.sh_degree;
    return POTR_OK;
}

potr_status potr_codec_decode(const uint8_t* raw, size_t raw_bytes, float* means, float* scales, float* quats,
                              float* opacities, float* sh) {
#pragma clang fp contract(off)
    Header h;
    if (!read_header(raw, raw_bytes, h)) return fail(POTR_EINVAL, "not a bitstream of this codec");
    const int64_t N = (int64_t)h.n;
    if (N > 0 && (!means || !scales || !quats || !opacities || !sh)) return fail(POTR_EINVAL, "NULL buffer");
    const int D = (int)h.depth;
    const uint8_t* nodes = raw + sizeof(Header);
    const uint8_t* capsb = nodes + h.n_nodes;
    const uint8_t* stb = capsb + 4 * h.n_caps;   // int32 streams (not necessarily 4-byte aligned)
    auto st_at = [&](int64_t idx) {
        int32_t v;
        std::memcpy(&v, stb + 4 * idx, 4);
        return v;
    };
    // depth-first walk of the bytes: the leaves' centres in order
    struct Frame {
        int depth;
        uint32_t cell[3];
        uint8_t byte;
        int next;   // next octant to visit
    };
    Frame stack[24];
    int sp = -1;
    uint64_t pos = 0, ci = 0;
    int64_t out = 0;
    auto emit_leaf = [&](int depth, const uint32_t* cell) -> bool {
        uint32_t count = 1;
        if (depth == D) {
            if (ci >= h.n_caps) return false;
            std::memcpy(&count, capsb + 4 * ci, 4);
            ++ci;
        }
        const double step = h.size * std::ldexp(1.0, -depth);
        float c[3];
        for (int a = 0; a < 3; ++a) c[a] = (float)(h.lo[a] + ((double)cell[a] + 0.5) * step);
        for (uint32_t r = 0; r < count; ++r) {
            if (out >= N) return false;
            for (int a = 0; a < 3; ++a) means[3 * out + a] = c[a];
            ++out;
        }
        return true;
    };
    bool okp = true;
    if (h.n_nodes > 0) {
        // the root
        const uint8_t b = nodes[pos++];
        const uint32_t zero[3] = {0u, 0u, 0u};
        if (b == 0) {
            okp = emit_leaf(0, zero);
        } else {
            stack[++sp] = Frame{0, {0u, 0u, 0u}, b, 0};
        }
        while (okp && sp >= 0) {
            Frame& f = stack[sp];
            while (f.next < 8 && !((f.byte >> f.next) & 1)) ++f.next;
            if (f.next == 8) {
                --sp;
                continue;
            }
            const int c = f.next++;
            const int cd = f.depth + 1;
            const uint32_t cell[3] = {2 * f.cell[0] + (uint32_t)(c & 1), 2 * f.cell[1] + (uint32_t)((c >> 1) & 1),
                                      2 * f.cell[2] + (uint32_t)((c >> 2) & 1)};
            if (pos >= h.n_nodes || cd > D) {
                okp = false;
                break;
            }
            const uint8_t b2 = nodes[pos++];
            if (b2 == 0) {
                okp = emit_leaf(cd, cell);
            } else {
                if (cd == D) {
                    okp = false;
                    break;
                }
                stack[++sp] = Frame{cd, {cell[0], cell[1], cell[2]}, b2, 0};
            }
        }
    }
    if (!okp || pos != h.n_nodes || ci != h.n_caps || out != N) return fail(POTR_EINVAL, "octree bytes do not parse");
    const double sf_scale = h.sf[0], sf_rot = h.sf[1], sf_opac = h.sf[2], sf_sh = h.sf[3];
    const int nsh = ((int)h.sh_degree + 1) * ((int)h.sh_degree + 1);
    int64_t dc[3] = {0, 0, 0};
    for (int64_t k = 0; k < N; ++k) {
        opacities[k] = (float)(((double)st_at(k) + 0.25) / sf_opac);
        for (int a = 0; a < 3; ++a) scales[3 * k + a] = (float)((double)st_at((1 + a) * N + k) / sf_scale);
        double x[3];
        for (int a = 0; a < 3; ++a) x[a] = (double)st_at((4 + a) * N + k) / sf_rot;
        const double n2 = (x[0] * x[0] + x[1] * x[1]) + x[2] * x[2];
        const double r = 1.0 - n2;
        quats[4 * k] = (float)std::sqrt(r > 0.0 ? r : 0.0);
        for (int a = 0; a < 3; ++a) quats[4 * k + 1 + a] = (float)x[a];
        float* o = sh + 48 * k;
        for (int j = 0; j < 16; ++j)
            for (int ch = 0; ch < 3; ++ch) {
                float v = 0.f;
                if (j < nsh) {
                    int64_t q = st_at((int64_t)(7 + 3 * j + ch) * N + k);
                    if (j == 0) {
                        dc[ch] += q;
                        q = dc[ch];
                    }
                    v = (float)((double)q / sf_sh);
                }
                o[3 * j + ch] = v;
            }
    }
    return POTR_OK;
}

}  // extern "C"
