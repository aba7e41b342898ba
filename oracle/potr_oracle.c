/*
 * FP64 CPU oracle for the POTR removal-effect rasterizer -- TEST INFRASTRUCTURE ONLY.
 * Loaded only by tests, the smoke check and the benchmark's CPU-baseline leg;
 * the HIP path never calls it and shares no code with it.
 *
 * Readings adopted where the paper is silent (each is also a field of orc_config):
 *  - pinhole u = fx*x/z + cx, pixel (i, j) samples (i + 0.5, j + 0.5);
 *  - the affine approximation is the Jacobian of the pinhole map at the centre,
 *    with x/z, y/z clamped to +-jclamp times the half field of view, plus an
 *    eps2d low-pass on the 2D covariance diagonal;
 *  - covariance Sigma = R(q) diag(s^2) R(q)^T with q = (w, x, y, z) normalised;
 *  - colour = max(0, sum_i L_i Y_i(d) + 1/2), d = unit vector from the camera
 *    centre to the splat centre, real SH with the Condon-Shortley phase;
 *  - a splat is blended at a pixel iff q <= q_max and o*exp(-q/2) >= alpha_min,
 *    with alpha = min(alpha_max, o*exp(-q/2)); the walk stops before the splat
 *    that would drive T below t_min (t_min = 0: no early stop);
 *  - background colour bg enters as T_final * bg.
 */
#define _GNU_SOURCE
#include "potr_oracle.h"

#include <math.h>
#include <pthread.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_version(void) { return 1; }

/* ------------------------------------------------------------------------- */
/* Real spherical harmonics (Sec. 3): Y_{l,m} from the associated Legendre     */
/* functions P_l^m (Condon-Shortley phase included) and                        */
/* K_l^m = sqrt((2l+1)/(4 pi) (l-|m|)!/(l+|m|)!):                              */
/*   m > 0: sqrt(2) K cos(m phi) P_l^m(cos theta)                              */
/*   m = 0: K P_l^0(cos theta)                                                 */
/*   m < 0: sqrt(2) K sin(|m| phi) P_l^|m|(cos theta)                          */
/* ------------------------------------------------------------------------- */
static double factorial(int n) { double f = 1.0; for (int i = 2; i <= n; ++i) f *= i; return f; }

static double legendre_p(int l, int m, double x) /* m >= 0, with (-1)^m phase */
{
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    double pmm = 1.0;                      /* P_m^m = (-1)^m (2m-1)!! s^m */
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pm1 = x * (2.0 * m + 1.0) * pmm; /* P_{m+1}^m */
    if (l == m + 1) return pm1;
    double pl = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pl = ((2.0 * ll - 1.0) * x * pm1 - (ll + m - 1.0) * pmm) / (ll - m);
        pmm = pm1;
        pm1 = pl;
    }
    return pl;
}

void orc_sh_basis(int32_t lmax, const double d[3], double* out)
{
    double ct = d[2];
    double phi = atan2(d[1], d[0]);
    for (int l = 0; l <= lmax; ++l) {
        for (int m = -l; m <= l; ++m) {
            int am = m < 0 ? -m : m;
            double K = sqrt((2.0 * l + 1.0) / (4.0 * M_PI) * factorial(l - am) / factorial(l + am));
            double P = legendre_p(l, am, ct);
            double y;
            if (m > 0) y = sqrt(2.0) * K * cos(m * phi) * P;
            else if (m == 0) y = K * P;
            else y = sqrt(2.0) * K * sin(am * phi) * P;
            out[l * (l + 1) + m] = y;
        }
    }
}

/* ------------------------------------------------------------------------- */
/* Projection (Sec. 3: affine approximation of the projective transform).      */
/* ------------------------------------------------------------------------- */
static void quat_rotation(const double qn[4], double M[9])
{
    double w = qn[0], x = qn[1], y = qn[2], z = qn[3];
    M[0] = 1 - 2 * (y * y + z * z); M[1] = 2 * (x * y - w * z);     M[2] = 2 * (x * z + w * y);
    M[3] = 2 * (x * y + w * z);     M[4] = 1 - 2 * (x * x + z * z); M[5] = 2 * (y * z - w * x);
    M[6] = 2 * (x * z - w * y);     M[7] = 2 * (y * z + w * x);     M[8] = 1 - 2 * (x * x + y * y);
}

/* Camera-space depth in FP32 by the fixed chain t_z + R20 x + R21 y + R22 z,
 * each step one fused multiply-add; its bits are the depth sort key. */
static float depth_f32(const orc_camera* cam, const double* m)
{
    float acc = cam->t[2];
    acc = fmaf(cam->R[6], (float)m[0], acc);
    acc = fmaf(cam->R[7], (float)m[1], acc);
    acc = fmaf(cam->R[8], (float)m[2], acc);
    return acc;
}

static void camera_eye(const orc_camera* cam, double eye[3])
{
    for (int i = 0; i < 3; ++i)
        eye[i] = -((double)cam->R[0 + i] * cam->t[0] + (double)cam->R[3 + i] * cam->t[1] +
                   (double)cam->R[6 + i] * cam->t[2]);
}

void orc_project(int64_t N, const orc_camera* cam, const orc_config* cfg,
                 const double* means, const double* scales, const double* quats,
                 const double* opac, const double* sh,
                 double* mean2d, double* cov2d, double* conic, double* rgb,
                 uint32_t* depth_key, int32_t* rect, int32_t* tiles_touched)
{
    const int W = cam->width, H = cam->height, tw = cfg->tile_w, th = cfg->tile_h;
    double eye[3];
    camera_eye(cam, eye);
    const int nsh = (cfg->sh_degree + 1) * (cfg->sh_degree + 1);
    for (int64_t i = 0; i < N; ++i) {
        const double* m = means + 3 * i;
        float z32 = depth_f32(cam, m);
        uint32_t key;
        memcpy(&key, &z32, 4);
        depth_key[i] = key;
        tiles_touched[i] = 0;
        for (int k = 0; k < 4; ++k) rect[4 * i + k] = 0;
        for (int k = 0; k < 2; ++k) mean2d[2 * i + k] = 0;
        for (int k = 0; k < 3; ++k) { cov2d[3 * i + k] = 0; conic[3 * i + k] = 0; rgb[3 * i + k] = 0; }

        /* camera-space centre */
        double p[3];
        for (int r = 0; r < 3; ++r)
            p[r] = (double)cam->R[3 * r] * m[0] + (double)cam->R[3 * r + 1] * m[1] +
                   (double)cam->R[3 * r + 2] * m[2] + (double)cam->t[r];
        if (!(z32 > cfg->near_z)) continue;
        double o = opac[i];
        if (!(o >= (double)cfg->alpha_min)) continue;

        /* 3D covariance from scale and rotation */
        const double* q = quats + 4 * i;
        double qn2 = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
        if (!(qn2 > 0.0)) continue;
        double qinv = 1.0 / sqrt(qn2), qn[4];
        for (int k = 0; k < 4; ++k) qn[k] = q[k] * qinv;
        double Rq[9];
        quat_rotation(qn, Rq);
        double s2[3];
        for (int k = 0; k < 3; ++k) s2[k] = scales[3 * i + k] * scales[3 * i + k];
        double Sig[9];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += Rq[3 * a + k] * s2[k] * Rq[3 * b + k];
                Sig[3 * a + b] = acc;
            }
        /* Jacobian of the pinhole map at the centre, camera rotation folded in */
        double z = p[2];
        double limx = (double)cfg->jclamp * 0.5 * W / cam->fx;
        double limy = (double)cfg->jclamp * 0.5 * H / cam->fy;
        double tx = fmin(limx, fmax(-limx, p[0] / z));
        double ty = fmin(limy, fmax(-limy, p[1] / z));
        double J[6] = { cam->fx / z, 0.0, -cam->fx * tx / z,
                        0.0, cam->fy / z, -cam->fy * ty / z };
        double T[6]; /* T = J * Rcam */
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 3; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k) acc += J[3 * a + k] * (double)cam->R[3 * k + b];
                T[3 * a + b] = acc;
            }
        double C2[4];
        for (int a = 0; a < 2; ++a)
            for (int b = 0; b < 2; ++b) {
                double acc = 0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += T[3 * a + k] * Sig[3 * k + l] * T[3 * b + l];
                C2[2 * a + b] = acc;
            }
        double cxx = C2[0] + cfg->eps2d, cxy = 0.5 * (C2[1] + C2[2]), cyy = C2[3] + cfg->eps2d;
        double det = cxx * cyy - cxy * cxy;
        if (!(det > 0.0)) continue;
        double u = cam->fx * p[0] / z + cam->cx;
        double v = cam->fy * p[1] / z + cam->cy;

        /* conservative pixel rectangle: AABB of the ellipse q <= t_cut */
        double t_cut = fmin((double)cfg->q_max, 2.0 * log(o / (double)cfg->alpha_min));
        double rx = sqrt(t_cut * cxx) * (1.0 + 1.0 / 1024.0) + 1.0 / 64.0;
        double ry = sqrt(t_cut * cyy) * (1.0 + 1.0 / 1024.0) + 1.0 / 64.0;
        if (!isfinite(u) || !isfinite(v) || !isfinite(rx) || !isfinite(ry)) continue;
        double ilo = fmax(ceil(u - rx - 0.5), 0.0), ihi = fmin(floor(u + rx - 0.5), W - 1.0);
        double jlo = fmax(ceil(v - ry - 0.5), 0.0), jhi = fmin(floor(v + ry - 0.5), H - 1.0);

        mean2d[2 * i] = u;
        mean2d[2 * i + 1] = v;
        cov2d[3 * i] = cxx; cov2d[3 * i + 1] = cxy; cov2d[3 * i + 2] = cyy;
        conic[3 * i] = cyy / det; conic[3 * i + 1] = -cxy / det; conic[3 * i + 2] = cxx / det;

        /* colour from SH along the camera -> centre direction */
        double d[3] = { m[0] - eye[0], m[1] - eye[1], m[2] - eye[2] };
        double dn = sqrt(d[0] * d[0] + d[1] * d[1] + d[2] * d[2]);
        for (int k = 0; k < 3; ++k) d[k] /= dn;
        double Y[16];
        orc_sh_basis(cfg->sh_degree, d, Y);
        for (int c = 0; c < 3; ++c) {
            double acc = 0.0;
            for (int k = 0; k < nsh; ++k) acc += sh[48 * i + 3 * k + c] * Y[k];
            rgb[3 * i + c] = fmax(0.0, acc + 0.5);
        }
        if (!(ilo <= ihi) || !(jlo <= jhi)) continue;
        int x0 = (int)ilo / tw, x1 = (int)ihi / tw + 1, y0 = (int)jlo / th, y1 = (int)jhi / th + 1;
        rect[4 * i] = x0; rect[4 * i + 1] = y0; rect[4 * i + 2] = x1; rect[4 * i + 3] = y1;
        tiles_touched[i] = (x1 - x0) * (y1 - y0);
    }
}

/* ------------------------------------------------------------------------- */
/* Tile lists ordered by (tile, depth key, splat id).                          */
/* ------------------------------------------------------------------------- */
typedef struct { uint32_t tile, key, id; } orc_pair;

static int pair_cmp(const void* a, const void* b)
{
    const orc_pair* x = (const orc_pair*)a;
    const orc_pair* y = (const orc_pair*)b;
    if (x->tile != y->tile) return x->tile < y->tile ? -1 : 1;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->id != y->id) return x->id < y->id ? -1 : 1;
    return 0;
}

int64_t orc_bin_sort(int64_t N, int32_t tiles_x, int32_t tiles_y, const int32_t* rect,
                     const uint32_t* depth_key, int32_t* out_tile, int32_t* out_id,
                     int32_t* tile_ranges)
{
    int64_t n = 0;
    for (int64_t i = 0; i < N; ++i) {
        const int32_t* r = rect + 4 * i;
        if (r[2] > r[0] && r[3] > r[1]) n += (int64_t)(r[2] - r[0]) * (r[3] - r[1]);
    }
    if (!out_id) return n;
    orc_pair* pairs = (orc_pair*)malloc((size_t)(n > 0 ? n : 1) * sizeof(orc_pair));
    int64_t k = 0;
    for (int64_t i = 0; i < N; ++i) {
        const int32_t* r = rect + 4 * i;
        for (int ty = r[1]; ty < r[3]; ++ty)
            for (int tx = r[0]; tx < r[2]; ++tx) {
                pairs[k].tile = (uint32_t)(ty * tiles_x + tx);
                pairs[k].key = depth_key[i];
                pairs[k].id = (uint32_t)i;
                ++k;
            }
    }
    qsort(pairs, (size_t)n, sizeof(orc_pair), pair_cmp);
    int64_t T = (int64_t)tiles_x * tiles_y;
    for (int64_t t = 0; t < 2 * T; ++t) tile_ranges[t] = 0;
    for (int64_t j = 0; j < n; ++j) {
        if (out_tile) out_tile[j] = (int32_t)pairs[j].tile;
        out_id[j] = (int32_t)pairs[j].id;
        uint32_t t = pairs[j].tile;
        if (j == 0 || pairs[j - 1].tile != t) tile_ranges[2 * t] = (int32_t)j;
        if (j == n - 1 || pairs[j + 1].tile != t) tile_ranges[2 * t + 1] = (int32_t)(j + 1);
    }
    free(pairs);
    return n;
}

/* ------------------------------------------------------------------------- */
/* Work splitting over image rows (pthreads).                                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    void (*fn)(void* ctx, int row);
    void* ctx;
    int rows;
    int next;
    pthread_mutex_t mu;
} row_pool;

static void* row_worker(void* arg)
{
    row_pool* p = (row_pool*)arg;
    for (;;) {
        pthread_mutex_lock(&p->mu);
        int r = p->next++;
        pthread_mutex_unlock(&p->mu);
        if (r >= p->rows) break;
        p->fn(p->ctx, r);
    }
    return NULL;
}

static void parallel_rows(int rows, int n_threads, void (*fn)(void*, int), void* ctx)
{
    row_pool p;
    p.fn = fn; p.ctx = ctx; p.rows = rows; p.next = 0;
    pthread_mutex_init(&p.mu, NULL);
    if (n_threads < 1) n_threads = 1;
    if (n_threads > 256) n_threads = 256;
    pthread_t th[256];
    for (int t = 1; t < n_threads; ++t) pthread_create(&th[t], NULL, row_worker, &p);
    row_worker(&p);
    for (int t = 1; t < n_threads; ++t) pthread_join(th[t], NULL);
    pthread_mutex_destroy(&p.mu);
}

static void atomic_add_f64(double* addr, double v)
{
    double old;
    __atomic_load(addr, &old, __ATOMIC_RELAXED);
    for (;;) {
        double nw = old + v;
        if (__atomic_compare_exchange(addr, &old, &nw, 1, __ATOMIC_RELAXED, __ATOMIC_RELAXED)) return;
    }
}

/* ------------------------------------------------------------------------- */
/* Compositing (Sec. 3) and the removal effect (Sec. 4.2).                     */
/* ------------------------------------------------------------------------- */
typedef struct {
    int64_t N;
    const orc_camera* cam;
    const orc_config* cfg;
    const double *mean2d, *conic, *rgb;
    const double* opac;
    const int32_t *tile_ranges, *sorted_id;
    const float* target;
    int removal_method;
    int rec32;                  /* evaluate records rounded to FP32 (the stored record precision) */
    double *image, *p_final, *t_final;
    int32_t *n_walk, *n_blend;
    double *score_l1, *score_se, *importance, *magnitude, *flag_mass;
    uint8_t* pixel_flag;
    int64_t skip_id;            /* orc_render_without: the deleted splat, else -1 */
    int max_list;
    int64_t n_flagged;
    pthread_mutex_t mu;
} render_ctx;

static inline double rec(const render_ctx* c, double x) { return c->rec32 ? (double)(float)x : x; }

/* One evaluation of splat s at pixel centre (px, py): q and o*G. */
static void eval_splat(const render_ctx* c, int64_t s, double px, double py,
                       double* q_out, double* dq_err, double* a0_out)
{
    const double mx = rec(c, c->mean2d[2 * s]), my = rec(c, c->mean2d[2 * s + 1]);
    double dx = px - mx, dy = py - my;
    double A = rec(c, c->conic[3 * s]), B = rec(c, c->conic[3 * s + 1]), C = rec(c, c->conic[3 * s + 2]);
    double q = A * dx * dx + 2.0 * B * dx * dy + C * dy * dy;
    *q_out = q;
    *a0_out = c->opac[s] * exp(-0.5 * q);
    /* Error bound of an FP32 evaluation of q from FP32-rounded inputs (used only
     * to flag decisions that FP32 arithmetic could take the other way): rounding
     * of the pixel offsets, of the conic and of the quadratic form itself. */
    const double u = ldexp(1.0, -24);
    double edx = c->rec32 ? fabs(dx) * u : (fabs(mx) + fabs(dx) + fabs(px)) * u;
    double edy = c->rec32 ? fabs(dy) * u : (fabs(my) + fabs(dy) + fabs(py)) * u;
    double qabs = fabs(A) * dx * dx + 2.0 * fabs(B * dx * dy) + fabs(C) * dy * dy;
    *dq_err = 2.0 * fabs(A * dx + B * dy) * edx + 2.0 * fabs(B * dx + C * dy) * edy + 12.0 * u * qabs;
}

/* A decision an FP32 evaluation could take the other way, and what it moves:
 * kind 0: splat at blended position `pos` is near a visibility threshold;
 * kind 1: a splat the oracle skips is near visible (it would sit before `pos`);
 * kind 2: the early stop is near its threshold; `dS` is what the splats an FP32
 *         walk might still blend add to the colour.
 * `imp` (set when the pixel is done) bounds the change of the pixel's colour
 * (L1 over channels) if the decision flips: the splat's own term T a |c|_1 plus,
 * since every later transmittance scales by (1 - a) or 1 / (1 - a) (Sec. 3,
 * T_k = prod_{j<k} (1 - a_j)), a / (1 - a) times what lies behind it,
 * |P_K - P_pos|_1 + T_K |bg|_1; for a stop, what an FP32 walk might still blend
 * plus the background seen at the stop, T |bg|_1. */
typedef struct { int kind, pos; double alpha, T, dS, imp; } flip_event;

/* A pixel is flagged (left out of image comparisons) when the decisions near a
 * threshold could together move its colour by this much: half the 1e-4 image
 * tolerance, so an unflagged pixel stays within it whichever way FP32 takes them. */
#define ORC_FLAG_IMAGE 5e-5

static void render_row(void* vctx, int py_i)
{
    render_ctx* c = (render_ctx*)vctx;
    const orc_camera* cam = c->cam;
    const orc_config* cfg = c->cfg;
    const int W = cam->width, tw = cfg->tile_w, th = cfg->tile_h;
    const int tiles_x = (W + tw - 1) / tw;
    const double qmax = cfg->q_max, amin = cfg->alpha_min, amax = cfg->alpha_max, tmin = cfg->t_min;
    const double bg[3] = { cfg->bg[0], cfg->bg[1], cfg->bg[2] };
    const double u = ldexp(1.0, -24);
    const int M = c->max_list + 1;
    double* al = (double*)malloc(sizeof(double) * M);
    double* Tk = (double*)malloc(sizeof(double) * M);
    double* Pk = (double*)malloc(sizeof(double) * 3 * (M + 1)); /* P_i, i = 0..K */
    int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * M);
    flip_event* ev = (flip_event*)malloc(sizeof(flip_event) * (M + 1));
    int64_t* extra_id = (int64_t*)malloc(sizeof(int64_t) * M);   /* splats blended only by a flip */
    double* extra_m = (double*)malloc(sizeof(double) * M);       /* ... their own term T a |c|_1 */
    double* extra_r = (double*)malloc(sizeof(double) * M);       /* ... a / (1 - a) */
    double* extra_b = (double*)malloc(sizeof(double) * M);       /* ... colour behind them (<0: P_K - P_pos) */
    int* extra_p = (int*)malloc(sizeof(int) * M);                /* ... blended position they would take */
    const int analyse = c->flag_mass != NULL || c->pixel_flag != NULL;
    const double sum_bg = fabs(bg[0]) + fabs(bg[1]) + fabs(bg[2]);
    int64_t row_flagged = 0;

    for (int px_i = 0; px_i < W; ++px_i) {
        const double px = px_i + 0.5, py = py_i + 0.5;
        const int tile = (py_i / th) * tiles_x + px_i / tw;
        const int beg = c->tile_ranges[2 * tile], end = c->tile_ranges[2 * tile + 1];
        double T = 1.0, elnT = 0.0;
        int K = 0, stop = end, n_ev = 0, n_extra = 0;
        Pk[0] = Pk[1] = Pk[2] = 0.0;
        int pos;
        for (pos = beg; pos < end; ++pos) {
            int64_t s = c->sorted_id[pos];
            if (s == c->skip_id) continue;
            double q, eq, a0;
            eval_splat(c, s, px, py, &q, &eq, &a0);
            double col[3];
            for (int ch = 0; ch < 3; ++ch) col[ch] = rec(c, c->rgb[3 * s + ch]);
            const double c1 = fabs(col[0]) + fabs(col[1]) + fabs(col[2]);
            /* decisions that an FP32 evaluation could flip (only looked for when
             * the flags or the allowance are asked for) */
            double elna = 0.5 * eq + 0.5 * q * 4.0 * u + 8.0 * u;
            const int vis_q = q <= qmax, vis_a = a0 >= amin;
            const int nq = analyse && fabs(q - qmax) <= 4.0 * eq;
            const int na = analyse && a0 > 0.0 && fabs(log(a0) - log(amin)) <= 4.0 * elna;
            const int may_flip = (nq && (vis_a || na)) || (na && (vis_q || nq));
            if (!vis_q || !vis_a) {
                if (may_flip) {
                    const double a = fmin(amax, a0);
                    flip_event e = { 1, K, a, T, T * a * c1, 0.0 };
                    ev[n_ev++] = e;
                    extra_id[n_extra] = s; extra_m[n_extra] = T * a * c1;
                    extra_r[n_extra] = a / (1.0 - a); extra_p[n_extra] = K; extra_b[n_extra++] = -1.0;
                }
                continue;
            }
            double a = fmin(amax, a0);
            double ea = a0 < amax ? elna : 0.0;
            double Tn = T * (1.0 - a);
            if (may_flip) {
                flip_event e = { 0, K, a, T, T * a * c1, 0.0 };
                ev[n_ev++] = e;
            }
            if (tmin > 0.0) {
                double e = elnT + a / (1.0 - a) * ea + 4.0 * u;
                int near_stop = analyse && fabs(log(Tn) - log(tmin)) <= 4.0 * e;
                if (near_stop) {
                    /* splats an FP32 walk could still blend from here on */
                    double Tv = T, dS = 0.0;
                    const int first_extra = n_extra;
                    for (int pv = pos; pv < end && n_extra < M; ++pv) {
                        int64_t sv = c->sorted_id[pv];
                        if (sv == c->skip_id) continue;
                        double qv, eqv, av;
                        eval_splat(c, sv, px, py, &qv, &eqv, &av);
                        if (!(qv <= qmax * (1.0 + 1e-3)) || !(av >= amin * (1.0 - 1e-3))) continue;
                        av = fmin(amax, av);
                        if (Tv * (1.0 - av) < tmin * exp(-8.0 * e)) break;
                        double cv[3];
                        for (int ch = 0; ch < 3; ++ch) cv[ch] = rec(c, c->rgb[3 * sv + ch]);
                        double m = Tv * av * (fabs(cv[0]) + fabs(cv[1]) + fabs(cv[2]));
                        dS += m;
                        if (Tn < tmin || pv > pos) {
                            extra_id[n_extra] = sv; extra_m[n_extra] = m;
                            extra_r[n_extra] = av / (1.0 - av); extra_p[n_extra] = K; extra_b[n_extra++] = 0.0;
                        }
                        Tv *= (1.0 - av);
                    }
                    for (int k = first_extra; k < n_extra; ++k) extra_b[k] = dS;
                    flip_event ee = { 2, K, a, T, dS, 0.0 };
                    ev[n_ev++] = ee;
                }
                if (Tn < tmin) { stop = pos; break; }
            }
            elnT += a / (1.0 - a) * ea + 4.0 * u;
            al[K] = a; Tk[K] = T; ids[K] = s;
            for (int ch = 0; ch < 3; ++ch) Pk[3 * (K + 1) + ch] = Pk[3 * K + ch] + T * a * col[ch];
            T = Tn;
            ++K;
        }
        if (pos >= end) stop = end;
        const int64_t pix = (int64_t)py_i * W + px_i;
        const double* PK = Pk + 3 * K;
        const double sumabsB = T * sum_bg;
        double imp = 0.0;
        for (int e = 0; e < n_ev; ++e) {
            flip_event* f = &ev[e];
            if (f->kind == 2) {
                f->imp = f->dS + f->T * sum_bg;
            } else {
                const double* Pp = Pk + 3 * f->pos;
                const double behind = fabs(PK[0] - Pp[0]) + fabs(PK[1] - Pp[1]) + fabs(PK[2] - Pp[2]);
                f->imp = f->dS + f->alpha / (1.0 - f->alpha) * (behind + sumabsB);
            }
            imp += f->imp;
        }
        const int flagged = imp >= ORC_FLAG_IMAGE;
        double img[3];
        for (int ch = 0; ch < 3; ++ch) img[ch] = PK[ch] + T * bg[ch];
        if (c->image) for (int ch = 0; ch < 3; ++ch) c->image[3 * pix + ch] = img[ch];
        if (c->p_final) for (int ch = 0; ch < 3; ++ch) c->p_final[3 * pix + ch] = PK[ch];
        if (c->t_final) c->t_final[pix] = T;
        if (c->n_walk) c->n_walk[pix] = stop;
        if (c->n_blend) c->n_blend[pix] = K;
        if (c->pixel_flag) c->pixel_flag[pix] = (uint8_t)flagged;
        row_flagged += flagged;

        const double sumabsP = fabs(PK[0]) + fabs(PK[1]) + fabs(PK[2]);
        for (int k = 0; k < K; ++k) {
            const double a = al[k];
            double col[3];
            for (int ch = 0; ch < 3; ++ch) col[ch] = rec(c, c->rgb[3 * ids[k] + ch]);
            double PD[3];
            if (c->removal_method == 0) {
                /* Sec. 4.2: PD_k = P_{i_k} - P_{i_k+1}/(1-a) + a/(1-a) P_K, plus the
                 * background term a/(1-a) T_K bg for a non-black background. */
                for (int ch = 0; ch < 3; ++ch)
                    PD[ch] = Pk[3 * k + ch] - Pk[3 * (k + 1) + ch] / (1.0 - a) + a / (1.0 - a) * PK[ch] +
                             a / (1.0 - a) * T * bg[ch];
            } else {
                /* definition: composite the blended list again without entry k */
                double Tw = 1.0, Cw[3] = { 0, 0, 0 };
                for (int j = 0; j < K; ++j) {
                    if (j == k) continue;
                    for (int ch = 0; ch < 3; ++ch) Cw[ch] += Tw * al[j] * rec(c, c->rgb[3 * ids[j] + ch]);
                    Tw *= (1.0 - al[j]);
                }
                for (int ch = 0; ch < 3; ++ch) PD[ch] = Cw[ch] + Tw * bg[ch] - img[ch];
            }
            int64_t s = ids[k];
            if (c->score_l1) atomic_add_f64(&c->score_l1[s], fabs(PD[0]) + fabs(PD[1]) + fabs(PD[2]));
            if (c->score_se && c->target) {
                double se = 0.0;
                for (int ch = 0; ch < 3; ++ch)
                    se += PD[ch] * PD[ch] + 2.0 * PD[ch] * (img[ch] - (double)c->target[3 * pix + ch]);
                atomic_add_f64(&c->score_se[s], se);
            }
            if (c->importance) atomic_add_f64(&c->importance[s], Tk[k] * a);
            const double ratio = a / (1.0 - a);
            const double own = Tk[k] * a * (fabs(col[0]) + fabs(col[1]) + fabs(col[2]));
            const double mag = own + ratio * (sumabsP + sumabsB);
            if (c->magnitude) atomic_add_f64(&c->magnitude[s], mag);
            /* a bound of |PD_k|_1 itself: T_k a |c_k|_1 + a/(1-a) (|S_k|_1 + T_K |bg|_1),
             * S_k = P_K - P_{k+1} */
            const double* P1 = Pk + 3 * (k + 1);
            const double pdb = own + ratio * (fabs(PK[0] - P1[0]) + fabs(PK[1] - P1[1]) + fabs(PK[2] - P1[2]) +
                                              sumabsB);
            if (n_ev > 0 && c->flag_mass) {
                /* first-order change of this splat's |PD| if an event flips */
                double F = 0.0;
                for (int e = 0; e < n_ev; ++e) {
                    const flip_event* f = &ev[e];
                    const double re = f->alpha / (1.0 - f->alpha);
                    if (f->kind == 2) {            /* early stop: k may vanish or S_k may grow */
                        if (k >= f->pos) F += pdb;
                        else F += ratio * f->imp;
                    } else if (f->kind == 0 && f->pos == k) {
                        F += pdb;                  /* its own visibility: PD_k may vanish */
                    } else if (f->pos > k) {       /* behind k: S_k and T_final move by at most imp */
                        F += ratio * f->imp;
                    } else {                       /* in front of k: PD_k scales by (1-a) or 1/(1-a) */
                        F += 2.0 * re * pdb;
                    }
                }
                atomic_add_f64(&c->flag_mass[s], 2.0 * F);
            }
        }
        if (n_ev > 0 && c->flag_mass) {
            for (int k = 0; k < n_extra; ++k) {
                double behind = extra_b[k];
                if (behind < 0.0) {
                    const double* Pp = Pk + 3 * extra_p[k];
                    behind = fabs(PK[0] - Pp[0]) + fabs(PK[1] - Pp[1]) + fabs(PK[2] - Pp[2]);
                }
                atomic_add_f64(&c->flag_mass[extra_id[k]], 2.0 * (extra_m[k] + extra_r[k] * (behind + sumabsB)));
            }
        }
    }
    free(al); free(Tk); free(Pk); free(ids); free(ev); free(extra_id); free(extra_m); free(extra_r); free(extra_b);
    free(extra_p);
    pthread_mutex_lock(&c->mu);
    c->n_flagged += row_flagged;
    pthread_mutex_unlock(&c->mu);
}

static int max_list_len(const orc_camera* cam, const orc_config* cfg, const int32_t* tile_ranges)
{
    int tiles = ((cam->width + cfg->tile_w - 1) / cfg->tile_w) * ((cam->height + cfg->tile_h - 1) / cfg->tile_h);
    int m = 0;
    for (int t = 0; t < tiles; ++t) {
        int l = tile_ranges[2 * t + 1] - tile_ranges[2 * t];
        if (l > m) m = l;
    }
    return m;
}

int64_t orc_render(int64_t N, const orc_camera* cam, const orc_config* cfg,
                   const double* mean2d, const double* conic, const double* rgb,
                   const double* opac, const int32_t* tile_ranges, const int32_t* sorted_id,
                   const float* target, int32_t removal_method, int32_t record_f32, int32_t n_threads,
                   double* image, double* p_final, double* t_final, int32_t* n_walk,
                   int32_t* n_blend, double* score_l1, double* score_se, double* importance,
                   double* magnitude, double* flag_mass, uint8_t* pixel_flag)
{
    render_ctx c;
    memset(&c, 0, sizeof(c));
    c.N = N; c.cam = cam; c.cfg = cfg; c.mean2d = mean2d; c.conic = conic; c.rgb = rgb; c.opac = opac;
    c.tile_ranges = tile_ranges; c.sorted_id = sorted_id; c.target = target;
    c.removal_method = removal_method;
    c.rec32 = record_f32;
    c.image = image; c.p_final = p_final; c.t_final = t_final; c.n_walk = n_walk; c.n_blend = n_blend;
    c.score_l1 = score_l1; c.score_se = score_se; c.importance = importance; c.magnitude = magnitude;
    c.flag_mass = flag_mass; c.pixel_flag = pixel_flag;
    c.skip_id = -1;
    c.max_list = max_list_len(cam, cfg, tile_ranges);
    pthread_mutex_init(&c.mu, NULL);
    parallel_rows(cam->height, n_threads, render_row, &c);
    pthread_mutex_destroy(&c.mu);
    return c.n_flagged;
}

void orc_render_without(int64_t N, const orc_camera* cam, const orc_config* cfg,
                        const double* mean2d, const double* conic, const double* rgb,
                        const double* opac, const int32_t* tile_ranges, const int32_t* sorted_id,
                        int64_t k, int32_t record_f32, double* image)
{
    render_ctx c;
    memset(&c, 0, sizeof(c));
    c.N = N; c.cam = cam; c.cfg = cfg; c.mean2d = mean2d; c.conic = conic; c.rgb = rgb; c.opac = opac;
    c.tile_ranges = tile_ranges; c.sorted_id = sorted_id;
    c.removal_method = 0;
    c.rec32 = record_f32;
    c.image = image;
    c.skip_id = k;
    c.max_list = max_list_len(cam, cfg, tile_ranges);
    pthread_mutex_init(&c.mu, NULL);
    parallel_rows(cam->height, 1, render_row, &c);
    pthread_mutex_destroy(&c.mu);
}

/* ------------------------------------------------------------------------- */
/* Backward: gradient of a loss L given dL/dC per pixel, through compositing   */
/* (Sec. 3) and the projection. Per pixel, C = P_k + T_k a_k c_k              */
/* + (S_k + T_K bg) / (1 - a_k) * (1 - a_k), so with S_k = P_K - P_{k+1}:       */
/*   dC/dc_k = T_k a_k,   dC/da_k = T_k c_k - (S_k + T_K bg) / (1 - a_k).       */
/* a_k = min(a_max, o G), G = exp(-q/2): zero gradient on the clamp.           */
/* ------------------------------------------------------------------------- */
typedef struct {
    const orc_camera* cam;
    const orc_config* cfg;
    const double *mean2d, *conic, *rgb, *opac;
    const int32_t *tile_ranges, *sorted_id;
    const double* dL_dC;
    double *g_mean2d, *g_conic, *g_opac, *g_rgb;
    int max_list;
} bwd_ctx;

static void backward_row(void* vctx, int py_i)
{
    bwd_ctx* c = (bwd_ctx*)vctx;
    const orc_camera* cam = c->cam;
    const orc_config* cfg = c->cfg;
    const int W = cam->width, tw = cfg->tile_w, th = cfg->tile_h;
    const int tiles_x = (W + tw - 1) / tw;
    const double qmax = cfg->q_max, amin = cfg->alpha_min, amax = cfg->alpha_max, tmin = cfg->t_min;
    const double bg[3] = { cfg->bg[0], cfg->bg[1], cfg->bg[2] };
    const int M = c->max_list + 1;
    double* al = (double*)malloc(sizeof(double) * M);
    double* a0s = (double*)malloc(sizeof(double) * M);
    double* Tk = (double*)malloc(sizeof(double) * M);
    double* dxs = (double*)malloc(sizeof(double) * 2 * M);
    double* Pk = (double*)malloc(sizeof(double) * 3 * (M + 1));
    int64_t* ids = (int64_t*)malloc(sizeof(int64_t) * M);
    for (int px_i = 0; px_i < W; ++px_i) {
        const double px = px_i + 0.5, py = py_i + 0.5;
        const int tile = (py_i / th) * tiles_x + px_i / tw;
        const int beg = c->tile_ranges[2 * tile], end = c->tile_ranges[2 * tile + 1];
        const int64_t pix = (int64_t)py_i * W + px_i;
        const double* g = c->dL_dC + 3 * pix;
        double T = 1.0;
        int K = 0;
        Pk[0] = Pk[1] = Pk[2] = 0.0;
        for (int pos = beg; pos < end; ++pos) {
            const int64_t s = c->sorted_id[pos];
            const double dx = px - c->mean2d[2 * s], dy = py - c->mean2d[2 * s + 1];
            const double A = c->conic[3 * s], B = c->conic[3 * s + 1], Cc = c->conic[3 * s + 2];
            const double q = A * dx * dx + 2.0 * B * dx * dy + Cc * dy * dy;
            const double a0 = c->opac[s] * exp(-0.5 * q);
            if (!(q <= qmax) || !(a0 >= amin)) continue;
            const double a = fmin(amax, a0);
            const double Tn = T * (1.0 - a);
            if (tmin > 0.0 && Tn < tmin) break;
            al[K] = a; a0s[K] = a0; Tk[K] = T; ids[K] = s; dxs[2 * K] = dx; dxs[2 * K + 1] = dy;
            for (int ch = 0; ch < 3; ++ch) Pk[3 * (K + 1) + ch] = Pk[3 * K + ch] + T * a * c->rgb[3 * s + ch];
            T = Tn;
            ++K;
        }
        const double* PK = Pk + 3 * K;
        for (int k = 0; k < K; ++k) {
            const int64_t s = ids[k];
            const double a = al[k];
            double dLda = 0.0;
            for (int ch = 0; ch < 3; ++ch) {
                const double S = PK[ch] - Pk[3 * (k + 1) + ch];
                dLda += g[ch] * (Tk[k] * c->rgb[3 * s + ch] - (S + T * bg[ch]) / (1.0 - a));
                atomic_add_f64(&c->g_rgb[3 * s + ch], g[ch] * Tk[k] * a);
            }
            if (a0s[k] >= amax) continue;           /* clamped: alpha does not move */
            const double o = c->opac[s];
            atomic_add_f64(&c->g_opac[s], dLda * a0s[k] / o);
            const double dLdq = -0.5 * a0s[k] * dLda;
            const double dx = dxs[2 * k], dy = dxs[2 * k + 1];
            const double A = c->conic[3 * s], B = c->conic[3 * s + 1], Cc = c->conic[3 * s + 2];
            /* dx = px - mean_x, so dq/dmean_x = -2 (A dx + B dy) */
            atomic_add_f64(&c->g_mean2d[2 * s], dLdq * -2.0 * (A * dx + B * dy));
            atomic_add_f64(&c->g_mean2d[2 * s + 1], dLdq * -2.0 * (B * dx + Cc * dy));
            atomic_add_f64(&c->g_conic[3 * s], dLdq * dx * dx);
            atomic_add_f64(&c->g_conic[3 * s + 1], dLdq * 2.0 * dx * dy);
            atomic_add_f64(&c->g_conic[3 * s + 2], dLdq * dy * dy);
        }
    }
    free(al); free(a0s); free(Tk); free(dxs); free(Pk); free(ids);
}

/* Derivative of d -> Y(d / |d|) at a unit direction, by a fourth-order central
 * difference of the recurrence-based basis: D[k*3 + j] = dY_k / du_j. */
static void sh_direction_jacobian(int lmax, const double d[3], double* D)
{
    const int nk = (lmax + 1) * (lmax + 1);
    const double h = 1e-3;
    const double w[4] = { 1.0, -8.0, 8.0, -1.0 }, off[4] = { -2.0, -1.0, 1.0, 2.0 };
    double Y[16];
    for (int k = 0; k < 3 * nk; ++k) D[k] = 0.0;
    for (int j = 0; j < 3; ++j) {
        for (int t = 0; t < 4; ++t) {
            double u[3] = { d[0], d[1], d[2] };
            u[j] += off[t] * h;
            const double n = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
            for (int i = 0; i < 3; ++i) u[i] /= n;
            orc_sh_basis(lmax, u, Y);
            for (int k = 0; k < nk; ++k) D[3 * k + j] += w[t] * Y[k] / (12.0 * h);
        }
    }
}

static void project_backward(int64_t i, const orc_camera* cam, const orc_config* cfg,
                             const double* means, const double* scales, const double* quats,
                             const double* opac, const double* sh,
                             const double* g_mean2d, const double* g_conic, const double* g_opac,
                             const double* g_rgb,
                             double* d_means, double* d_scales, double* d_quats, double* d_opac, double* d_sh)
{
    const double* m = means + 3 * i;
    const int W = cam->width, H = cam->height;
    double Rc[9], t[3];
    for (int k = 0; k < 9; ++k) Rc[k] = cam->R[k];
    for (int k = 0; k < 3; ++k) t[k] = cam->t[k];
    double p[3];
    for (int r = 0; r < 3; ++r) p[r] = Rc[3 * r] * m[0] + Rc[3 * r + 1] * m[1] + Rc[3 * r + 2] * m[2] + t[r];
    const double x = p[0], y = p[1], z = p[2], fx = cam->fx, fy = cam->fy;
    /* forward intermediates */
    const double* q = quats + 4 * i;
    const double qn = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    const double qh[4] = { q[0] / qn, q[1] / qn, q[2] / qn, q[3] / qn };
    double Rq[9];
    quat_rotation(qh, Rq);
    const double s[3] = { scales[3 * i], scales[3 * i + 1], scales[3 * i + 2] };
    double Mm[9], Sig[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) Mm[3 * r + k] = Rq[3 * r + k] * s[k];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += Mm[3 * a + k] * Mm[3 * b + k];
            Sig[3 * a + b] = acc;
        }
    const double limx = (double)cfg->jclamp * 0.5 * W / fx, limy = (double)cfg->jclamp * 0.5 * H / fy;
    const double rx = x / z, ry = y / z;
    const int freex = rx > -limx && rx < limx, freey = ry > -limy && ry < limy;
    const double tx = fmin(limx, fmax(-limx, rx)), ty = fmin(limy, fmax(-limy, ry));
    const double J[6] = { fx / z, 0.0, -fx * tx / z, 0.0, fy / z, -fy * ty / z };
    double T[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += J[3 * a + k] * Rc[3 * k + b];
            T[3 * a + b] = acc;
        }
    double C2[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k)
                for (int l = 0; l < 3; ++l) acc += T[3 * a + k] * Sig[3 * k + l] * T[3 * b + l];
            C2[2 * a + b] = acc;
        }
    C2[0] += cfg->eps2d;
    C2[3] += cfg->eps2d;
    C2[1] = C2[2] = 0.5 * (C2[1] + C2[2]);
    const double det = C2[0] * C2[3] - C2[1] * C2[2];
    const double Q[4] = { C2[3] / det, -C2[1] / det, -C2[2] / det, C2[0] / det };

    /* conic -> 2D covariance: dL/dSigma' = -Q G_Q Q, G_Q symmetric with the
     * off-diagonal gradient split over both entries */
    const double GQ[4] = { g_conic[3 * i], 0.5 * g_conic[3 * i + 1], 0.5 * g_conic[3 * i + 1], g_conic[3 * i + 2] };
    double tmp[4], GS[4];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) tmp[2 * a + b] = GQ[2 * a] * Q[b] + GQ[2 * a + 1] * Q[2 + b];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 2; ++b) GS[2 * a + b] = -(Q[2 * a] * tmp[b] + Q[2 * a + 1] * tmp[2 + b]);
    /* Sigma' = T Sigma T^T: dL/dSigma = T^T GS T, dL/dT = 2 GS T Sigma */
    double GSig[9], GT[6], TS[6];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 2; ++k)
                for (int l = 0; l < 2; ++l) acc += T[3 * k + a] * GS[2 * k + l] * T[3 * l + b];
            GSig[3 * a + b] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += T[3 * a + k] * Sig[3 * k + b];
            TS[3 * a + b] = acc;
        }
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) GT[3 * a + b] = 2.0 * (GS[2 * a] * TS[b] + GS[2 * a + 1] * TS[3 + b]);
    /* T = J R: dL/dJ = GT R^T */
    double GJ[6];
    for (int a = 0; a < 2; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += GT[3 * a + k] * Rc[3 * b + k];
            GJ[3 * a + b] = acc;
        }
    /* J and the pixel centre as functions of the camera-space point */
    double gp[3] = { 0, 0, 0 };
    gp[2] += GJ[0] * (-fx / (z * z)) + GJ[4] * (-fy / (z * z));
    gp[0] += GJ[2] * (freex ? -fx / (z * z) : 0.0);
    gp[2] += GJ[2] * fx * tx / (z * z) * (freex ? 2.0 : 1.0);
    gp[1] += GJ[5] * (freey ? -fy / (z * z) : 0.0);
    gp[2] += GJ[5] * fy * ty / (z * z) * (freey ? 2.0 : 1.0);
    const double gu = g_mean2d[2 * i], gv = g_mean2d[2 * i + 1];
    gp[0] += gu * fx / z;
    gp[1] += gv * fy / z;
    gp[2] += -gu * fx * x / (z * z) - gv * fy * y / (z * z);
    for (int j = 0; j < 3; ++j) d_means[3 * i + j] += Rc[j] * gp[0] + Rc[3 + j] * gp[1] + Rc[6 + j] * gp[2];

    /* Sigma = M M^T, M = R(q) diag(s) */
    double GM[9];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            double acc = 0;
            for (int k = 0; k < 3; ++k) acc += (GSig[3 * a + k] + GSig[3 * k + a]) * Mm[3 * k + b];
            GM[3 * a + b] = acc;
        }
    double GR[9];
    for (int r = 0; r < 3; ++r)
        for (int k = 0; k < 3; ++k) {
            d_scales[3 * i + k] += GM[3 * r + k] * Rq[3 * r + k];
            GR[3 * r + k] = GM[3 * r + k] * s[k];
        }
    const double w = qh[0], X = qh[1], Y = qh[2], Z = qh[3];
    /* partial derivatives of the rotation entries w.r.t. (w, x, y, z) */
    const double dRw[9] = { 0, -2 * Z, 2 * Y, 2 * Z, 0, -2 * X, -2 * Y, 2 * X, 0 };
    const double dRx[9] = { 0, 2 * Y, 2 * Z, 2 * Y, -4 * X, -2 * w, 2 * Z, 2 * w, -4 * X };
    const double dRy[9] = { -4 * Y, 2 * X, 2 * w, 2 * X, 0, 2 * Z, -2 * w, 2 * Z, -4 * Y };
    const double dRz[9] = { -4 * Z, -2 * w, 2 * X, 2 * w, -4 * Z, 2 * Y, 2 * X, 2 * Y, 0 };
    double gqh[4] = { 0, 0, 0, 0 };
    for (int k = 0; k < 9; ++k) {
        gqh[0] += GR[k] * dRw[k];
        gqh[1] += GR[k] * dRx[k];
        gqh[2] += GR[k] * dRy[k];
        gqh[3] += GR[k] * dRz[k];
    }
    const double dotq = gqh[0] * qh[0] + gqh[1] * qh[1] + gqh[2] * qh[2] + gqh[3] * qh[3];
    for (int k = 0; k < 4; ++k) d_quats[4 * i + k] += (gqh[k] - qh[k] * dotq) / qn;

    d_opac[i] += g_opac[i];

    /* colour: max(0, sum_k L_k Y_k(d) + 1/2), d = (mu - eye) / |mu - eye| */
    double eye[3];
    camera_eye(cam, eye);
    double u[3] = { m[0] - eye[0], m[1] - eye[1], m[2] - eye[2] };
    const double un = sqrt(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]);
    double d[3] = { u[0] / un, u[1] / un, u[2] / un };
    const int nk = (cfg->sh_degree + 1) * (cfg->sh_degree + 1);
    double Yb[16], D[48];
    orc_sh_basis(cfg->sh_degree, d, Yb);
    sh_direction_jacobian(cfg->sh_degree, d, D);
    double gY[16];
    for (int k = 0; k < nk; ++k) gY[k] = 0.0;
    for (int ch = 0; ch < 3; ++ch) {
        double pre = 0.5;
        for (int k = 0; k < nk; ++k) pre += sh[48 * i + 3 * k + ch] * Yb[k];
        if (!(pre > 0.0)) continue;
        const double gc = g_rgb[3 * i + ch];
        for (int k = 0; k < nk; ++k) {
            d_sh[48 * i + 3 * k + ch] += gc * Yb[k];
            gY[k] += gc * sh[48 * i + 3 * k + ch];
        }
    }
    for (int j = 0; j < 3; ++j) {
        double acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += gY[k] * D[3 * k + j];
        d_means[3 * i + j] += acc / un;
    }
}

void orc_backward(int64_t N, const orc_camera* cam, const orc_config* cfg,
                  const double* means, const double* scales, const double* quats,
                  const double* opac, const double* sh,
                  const double* mean2d, const double* conic, const double* rgb,
                  const int32_t* tile_ranges, const int32_t* sorted_id,
                  const double* dL_dimage, int32_t n_threads,
                  double* d_means, double* d_scales, double* d_quats, double* d_opac,
                  double* d_sh, double* d_mean2d, double* d_conic, double* d_rgb)
{
    double* g_mean2d = (double*)calloc((size_t)(2 * N + 1), sizeof(double));
    double* g_conic = (double*)calloc((size_t)(3 * N + 1), sizeof(double));
    double* g_opac = (double*)calloc((size_t)(N + 1), sizeof(double));
    double* g_rgb = (double*)calloc((size_t)(3 * N + 1), sizeof(double));
    bwd_ctx c;
    memset(&c, 0, sizeof(c));
    c.cam = cam; c.cfg = cfg; c.mean2d = mean2d; c.conic = conic; c.rgb = rgb; c.opac = opac;
    c.tile_ranges = tile_ranges; c.sorted_id = sorted_id; c.dL_dC = dL_dimage;
    c.g_mean2d = g_mean2d; c.g_conic = g_conic; c.g_opac = g_opac; c.g_rgb = g_rgb;
    c.max_list = max_list_len(cam, cfg, tile_ranges);
    parallel_rows(cam->height, n_threads, backward_row, &c);
    for (int64_t i = 0; i < N; ++i) {
        if (d_mean2d) { d_mean2d[2 * i] += g_mean2d[2 * i]; d_mean2d[2 * i + 1] += g_mean2d[2 * i + 1]; }
        if (d_conic) for (int k = 0; k < 3; ++k) d_conic[3 * i + k] += g_conic[3 * i + k];
        if (d_rgb) for (int k = 0; k < 3; ++k) d_rgb[3 * i + k] += g_rgb[3 * i + k];
        const int touched = g_mean2d[2 * i] != 0.0 || g_mean2d[2 * i + 1] != 0.0 || g_opac[i] != 0.0 ||
                            g_rgb[3 * i] != 0.0 || g_rgb[3 * i + 1] != 0.0 || g_rgb[3 * i + 2] != 0.0 ||
                            g_conic[3 * i] != 0.0 || g_conic[3 * i + 1] != 0.0 || g_conic[3 * i + 2] != 0.0;
        if (!touched) continue;
        project_backward(i, cam, cfg, means, scales, quats, opac, sh, g_mean2d, g_conic, g_opac, g_rgb,
                         d_means, d_scales, d_quats, d_opac, d_sh);
    }
    free(g_mean2d); free(g_conic); free(g_opac); free(g_rgb);
}
