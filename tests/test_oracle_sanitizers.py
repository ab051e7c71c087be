"""The C oracle under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only): a driver compiled with it calls every oracle entry point -- 1-3 d,
periodic and open boxes, both routes, every operator with its scales, threads
over rows, row subsets, finite differences, the dense sums and the time step --
and must finish with no sanitizer report.  Values are checked elsewhere; this
checks memory and arithmetic safety."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

DRIVER = r"""
#include "oracle.c"
#include <stdio.h>

static uint64_t st = 12345;
static double unif(void) { st = st * 6364136223846793005ULL + 1442695040888963407ULL; return (double)(st >> 11) * 0x1p-53; }

static int run_case(int d, const int* per, double L, double r, int n, int dtype, int nthreads) {
    double lo[3] = {0, 0, 0}, hi[3] = {L, L, L};
    int32_t pr[3] = {per[0], per[1], per[2]}, reach[3] = {1 + (n % 3), 1, 1};
    or_grid g;
    if (or_grid_init(&g, d, dtype, lo, hi, pr, r, NULL, reach) != OR_OK) return 1;
    double* x = malloc(sizeof(double) * n * d);
    double* a = malloc(sizeof(double) * n);
    double* gy = malloc(sizeof(double) * n * 3);
    for (int i = 0; i < n * d; ++i) { double v = unif() * L; if (dtype == OR_F32) v = (double)(float)v; if (v >= L) v = 0; x[i] = v; }
    for (int i = 0; i < n; ++i) a[i] = 0.2 + 0.3 * unif();
    for (int i = 0; i < n * 3; ++i) gy[i] = unif() - 0.5;
    uint32_t* ids = malloc(sizeof(uint32_t) * n);
    uint32_t* perm = malloc(sizeof(uint32_t) * n);
    uint32_t* off = malloc(sizeof(uint32_t) * (g.ncells + 1));
    or_cell_ids(&g, n, x, ids);
    or_sort_cells(&g, n, ids, perm, off);
    for (int route = 0; route < 2; ++route) {
        int64_t m = or_pairs(&g, route, n, x, 0, NULL, NULL);
        uint32_t* pi = malloc(sizeof(uint32_t) * (m + 1));
        uint32_t* pj = malloc(sizeof(uint32_t) * (m + 1));
        or_pairs(&g, route, n, x, m, pi, pj);
        free(pi); free(pj);
        int64_t rows[3] = {0, n / 2, n - 1};
        for (int op = 0; op <= 4; ++op) {
            double prm[4] = {0.7, 0, 0, 0};
            int ny = or_op_ny(op, d);
            const double* aa = op == OR_OP_DEM_SPRING ? a : NULL;
            double* y = malloc(sizeof(double) * n * ny);
            double* sc = malloc(sizeof(double) * n);
            double* cd = malloc(sizeof(double) * n);
            double* gx = malloc(sizeof(double) * n * d);
            double* ga = malloc(sizeof(double) * n);
            double* s4 = malloc(sizeof(double) * n * 4);
            or_pair_sum(&g, route, op, prm, n, x, aa, 0, NULL, y, sc, cd, nthreads);
            or_pair_sum(&g, route, op, prm, n, x, aa, 3, rows, y, NULL, NULL, 1);
            or_pair_sum_backward(&g, route, op, prm, n, x, aa, gy, 0, NULL, gx, ga, s4, s4 + n, s4 + 2 * n, s4 + 3 * n, nthreads);
            or_pair_sum_backward(&g, route, op, prm, n, x, aa, gy, 3, rows, gx, ga, NULL, NULL, NULL, NULL, 1);
            free(y); free(sc); free(cd); free(gx); free(ga); free(s4);
        }
    }
    int64_t coords[4] = {0, 1, (int64_t)n * d - 1, (int64_t)n * d};
    double fd[4];
    for (int op = 1; op <= 4; ++op) {
        double prm[4] = {0.7, 0, 0, 0};
        or_fd_grad(&g, op, prm, n, x, a, gy, op == OR_OP_DEM_SPRING ? 4 : 3, coords, 1e-6, fd);
    }
    (void)or_tie_band(&g, n, x);
    double* v = calloc((size_t)n * d, sizeof(double));
    double* sv = malloc(sizeof(double) * n);
    double* cv = malloc(sizeof(double) * n);
    if (d == 2 || d == 3) or_md_step(&g, 1, 1e-3, 1.0, n, x, v, sv, cv);
    double* yd = malloc(sizeof(double) * n);
    double* sd = malloc(sizeof(double) * n);
    int64_t drows[2] = {0, n - 1};
    or_dense_gauss(d, n, x, n, x, a, 0.3, 2, drows, yd, sd);
    for (int kind = 0; kind < 2; ++kind) {
        double* gxt = malloc(sizeof(double) * n * d);
        double* gxs = malloc(sizeof(double) * n * d);
        double* gw = malloc(sizeof(double) * n);
        double* s3 = malloc(sizeof(double) * n * 3);
        or_dense_sum(kind, 0.3, d, n, x, n, x, a, yd, sd);
        or_dense_backward(kind, 0.3, d, n, x, n, x, a, gy, gxt, gxs, gw, s3, s3 + n, s3 + 2 * n);
        free(gxt); free(gxs); free(gw); free(s3);
    }
    free(x); free(a); free(gy); free(ids); free(perm); free(off); free(v); free(sv); free(cv); free(yd); free(sd);
    return 0;
}

int main(void) {
    int p111[3] = {1, 1, 1}, p010[3] = {0, 1, 0}, p000[3] = {0, 0, 0};
    int bad = 0;
    bad |= run_case(1, p111, 20.0, 1.0, 300, OR_F32, 1);
    bad |= run_case(2, p111, 1.0, 0.1, 400, OR_F64, 3);
    bad |= run_case(2, p010, 3.0, 0.4, 350, OR_F32, 4);
    bad |= run_case(3, p111, 4.0, 1.0, 500, OR_F32, 2);
    bad |= run_case(3, p000, 3.0, 0.9, 257, OR_F64, 8);
    printf("done %d\n", bad);
    return bad;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracle_runs_clean_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-I", os.path.dirname(SRC),
           str(drv), "-o", str(exe), "-lm", "-lpthread"]
    subprocess.run(cmd, check=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and "done 0" in r.stdout, (r.returncode, r.stdout[-2000:], r.stderr[-4000:])
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-4000:]
