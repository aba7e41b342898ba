"""The oracle's C under AddressSanitizer and UndefinedBehaviorSanitizer (host code
only, gcc): one small scene through projection, tile lists, both compositing
methods, literal deletion and the backward, with no sanitizer report."""
import os
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(os.path.dirname(HERE), "oracle", "potr_oracle.c")

DRIVER = r"""
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "potr_oracle.h"

static unsigned long long s = 12345;
static double u(void) { s = s * 6364136223846793005ULL + 1442695040888963407ULL; return (double)(s >> 11) / 9007199254740992.0; }

int main(void) {
    const int64_t N = 300;
    const int W = 64, H = 48;
    double *m = malloc(N * 3 * 8), *sc = malloc(N * 3 * 8), *q = malloc(N * 4 * 8), *o = malloc(N * 8), *sh = malloc(N * 48 * 8);
    for (int64_t i = 0; i < N; ++i) {
        for (int a = 0; a < 3; ++a) { m[3 * i + a] = 2 * u() - 1; sc[3 * i + a] = 0.02 + 0.08 * u(); }
        for (int a = 0; a < 4; ++a) q[4 * i + a] = 2 * u() - 1;
        o[i] = 0.3 + 0.6 * u();
        for (int k = 0; k < 48; ++k) sh[48 * i + k] = (k < 3 ? 0.5 : 0.05) * (2 * u() - 1);
    }
    sc[0] = 3.0;                      /* one large splat over many tiles */
    m[3 * 5 + 2] = -3.5;              /* one behind the camera */
    orc_camera cam = {{1, 0, 0, 0, 1, 0, 0, 0, 1}, {0, 0, 3}, 55, 55, 32, 24, W, H};
    orc_config cfg = {16, 16, 0.3f, 0.2f, 1.3f, 1.0f / 255.0f, 0.99f, 9.0f, 1e-4f, {0.1f, 0.2f, 0.3f}, 3};
    double *m2 = malloc(N * 2 * 8), *cov = malloc(N * 3 * 8), *con = malloc(N * 3 * 8), *rgb = malloc(N * 3 * 8);
    uint32_t* key = malloc(N * 4);
    int32_t *rect = malloc(N * 4 * 4), *tt = malloc(N * 4);
    orc_project(N, &cam, &cfg, m, sc, q, o, sh, m2, cov, con, rgb, key, rect, tt);
    const int tx = (W + 15) / 16, ty = (H + 15) / 16;
    int64_t np = orc_bin_sort(N, tx, ty, rect, key, NULL, NULL, NULL);
    int32_t *tile = malloc((np + 1) * 4), *ids = malloc((np + 1) * 4), *rng = malloc(tx * ty * 2 * 4);
    orc_bin_sort(N, tx, ty, rect, key, tile, ids, rng);
    const int64_t P = (int64_t)W * H;
    double *img = calloc(P * 3, 8), *pf = calloc(P * 3, 8), *tf = calloc(P, 8);
    int32_t *nw = calloc(P, 4), *nb = calloc(P, 4);
    double *l1 = calloc(N, 8), *se = calloc(N, 8), *im = calloc(N, 8), *mag = calloc(N, 8), *fl = calloc(N, 8);
    uint8_t* pflag = calloc(P, 1);
    float* tgt = malloc(P * 3 * 4);
    for (int64_t k = 0; k < P * 3; ++k) tgt[k] = (float)u();
    for (int method = 0; method < 2; ++method)
        orc_render(N, &cam, &cfg, m2, con, rgb, o, rng, ids, tgt, method, 1, 2, img, pf, tf, nw, nb, l1, se, im, mag, fl, pflag);
    double* img2 = calloc(P * 3, 8);
    orc_render_without(N, &cam, &cfg, m2, con, rgb, o, rng, ids, 1, 1, img2);
    double* dl = malloc(P * 3 * 8);
    for (int64_t k = 0; k < P * 3; ++k) dl[k] = 1.0;
    double *dm = calloc(N * 3, 8), *ds = calloc(N * 3, 8), *dq = calloc(N * 4, 8), *dop = calloc(N, 8), *dsh = calloc(N * 48, 8);
    double *dm2 = calloc(N * 2, 8), *dcon = calloc(N * 3, 8), *drgb = calloc(N * 3, 8);
    orc_backward(N, &cam, &cfg, m, sc, q, o, sh, m2, con, rgb, rng, ids, dl, 2, dm, ds, dq, dop, dsh, dm2, dcon, drgb);
    double total = 0;
    for (int64_t i = 0; i < N; ++i) total += l1[i] + fabs(dm[3 * i]);
    printf("pairs %lld total %g\n", (long long)np, total);
    free(m); free(sc); free(q); free(o); free(sh); free(m2); free(cov); free(con); free(rgb); free(key); free(rect);
    free(tt); free(tile); free(ids); free(rng); free(img); free(pf); free(tf); free(nw); free(nb); free(l1); free(se);
    free(im); free(mag); free(fl); free(pflag); free(tgt); free(img2); free(dl); free(dm); free(ds); free(dq); free(dop);
    free(dsh); free(dm2); free(dcon); free(drgb);
    return np > 0 && total > 0 ? 0 : 3;
}
"""


def test_oracle_runs_clean_under_sanitizers(tmp_path):
    asan = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True).stdout.strip()
    if not os.path.isabs(asan) or not os.path.exists(asan):
        pytest.skip("gcc has no sanitizer runtime here")
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    subprocess.check_call(["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
                           "-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                           "-I", os.path.dirname(SRC), str(drv), SRC, "-o", str(exe), "-lm", "-lpthread"])
    # other preloaded libraries may come before the sanitizer runtime: allow that order
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-4000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
    assert r.stdout.startswith("pairs ")
