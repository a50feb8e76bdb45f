"""The oracle's C code under AddressSanitizer and UndefinedBehaviorSanitizer (host
code only, built with gcc): a driver exercises every entry point on a small jittered
lattice with every option on (correction tensor, artificial stress, XSPH, energy,
Tillotson, damage) and on the gravity tree, and any out-of-bounds access, leak, or
undefined operation fails the run."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import workloads as W

HERE = os.path.dirname(os.path.abspath(__file__))
ORACLE = os.path.join(os.path.dirname(HERE), "oracle")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>

int64_t orc_count_neighbours(int64_t, const double *, double, const int64_t *, int64_t, int64_t *);
void orc_fill_neighbours(int64_t, const double *, double, const int64_t *, int64_t, const int64_t *,
                         int32_t *);
void orc_prepass2(int64_t, const double *, const double *, const double *, const double *,
                  const double *, double *, double *, double *, double *);
void orc_eos(int64_t, const double *, const double *, const double *, double *, double *);
void orc_rhs2(int64_t, const double *, const double *, const double *, const double *,
              const double *, const double *, const double *, const double *, const int64_t *,
              int64_t, const int64_t *, const int32_t *, double *, double *, double *, double *,
              double *, double *, double *);
int64_t orc_gravity(int64_t, const double *, const double *, double, double, double,
                    const int64_t *, int64_t, double *, int64_t *, int32_t *);
int64_t orc_gravity_tree(int64_t, const double *, const double *, int64_t, int32_t *, int64_t *,
                         double *, double *);

static const double POS[] = {POS_VALUES};
static const double VEL[] = {VEL_VALUES};
static const double RHO[] = {RHO_VALUES};
static const double SS[] = {S_VALUES};
static const double M[] = {M_VALUES};
static const double U[] = {U_VALUES};
static const double D[] = {D_VALUES};
static const double PAR[] = {PAR_VALUES};
#define N NUM

static int finite_all(const double *a, int64_t k) {
    for (int64_t i = 0; i < k; ++i)
        if (!isfinite(a[i])) return 0;
    return 1;
}

int main(void) {
    const double h = PAR[0];
    int64_t *counts = malloc(N * sizeof(int64_t));
    const int64_t nnz = orc_count_neighbours(N, POS, h, NULL, 0, counts);
    int64_t *row_ptr = malloc((N + 1) * sizeof(int64_t));
    row_ptr[0] = 0;
    for (int i = 0; i < N; ++i) row_ptr[i + 1] = row_ptr[i] + counts[i];
    int32_t *col = malloc((nnz > 0 ? nnz : 1) * sizeof(int32_t));
    orc_fill_neighbours(N, POS, h, NULL, 0, row_ptr, col);

    double *p = malloc(N * sizeof(double)), *f = malloc(N * sizeof(double));
    double *cs = malloc(N * sizeof(double)), *sig = malloc(6 * N * sizeof(double));
    orc_prepass2(N, RHO, U, D, SS, PAR, p, f, cs, sig);
    orc_eos(N, RHO, U, PAR, p, cs);

    double *acc = malloc(3 * N * sizeof(double)), *drho = malloc(N * sizeof(double));
    double *dS = malloc(6 * N * sizeof(double)), *rs = malloc(N * sizeof(double));
    double *L = malloc(9 * N * sizeof(double)), *du = malloc(N * sizeof(double));
    double *xv = malloc(3 * N * sizeof(double));
    orc_rhs2(N, POS, VEL, RHO, U, D, SS, M, PAR, NULL, 0, row_ptr, col, acc, drho, dS, rs, L, du, xv);
    /* a target subset: every other particle */
    int64_t nt = N / 2;
    int64_t *tg = malloc(nt * sizeof(int64_t));
    for (int64_t t = 0; t < nt; ++t) tg[t] = 2 * t;
    int64_t *rp2 = malloc((nt + 1) * sizeof(int64_t));
    int64_t *c2 = malloc(nt * sizeof(int64_t));
    orc_count_neighbours(N, POS, h, tg, nt, c2);
    rp2[0] = 0;
    for (int64_t t = 0; t < nt; ++t) rp2[t + 1] = rp2[t] + c2[t];
    int32_t *col2 = malloc((rp2[nt] > 0 ? rp2[nt] : 1) * sizeof(int32_t));
    orc_fill_neighbours(N, POS, h, tg, nt, rp2, col2);
    orc_rhs2(N, POS, VEL, RHO, U, D, SS, M, PAR, tg, nt, rp2, col2, acc, drho, dS, rs, L, du, xv);

    double *ga = malloc(3 * N * sizeof(double));
    int64_t *gc = malloc(N * sizeof(int64_t));
    int32_t *gt = malloc(N * sizeof(int32_t));
    const int64_t nn = orc_gravity(N, POS, M, 1.0, 0.5, 0.01, NULL, 0, ga, gc, gt);
    orc_gravity(N, POS, M, 1.0, 0.0, 0.0, tg, nt, ga, gc, NULL);
    int32_t *dep = malloc(nn * sizeof(int32_t));
    int64_t *cor = malloc(3 * nn * sizeof(int64_t));
    double *gm = malloc(nn * sizeof(double)), *com = malloc(3 * nn * sizeof(double));
    orc_gravity_tree(N, POS, M, nn, dep, cor, gm, com);

    const int ok = finite_all(acc, 3 * nt) && finite_all(dS, 6 * nt) && finite_all(du, nt) &&
                   finite_all(xv, 3 * nt) && finite_all(ga, 3 * nt) && finite_all(sig, 6 * N) &&
                   finite_all(com, 3 * nn);
    free(counts); free(row_ptr); free(col); free(p); free(f); free(cs); free(sig);
    free(acc); free(drho); free(dS); free(rs); free(L); free(du); free(xv);
    free(tg); free(rp2); free(c2); free(col2); free(ga); free(gc); free(gt);
    free(dep); free(cor); free(gm); free(com);
    printf("driver %s: %lld partners, %lld inner nodes\n", ok ? "ok" : "NON-FINITE", (long long)nnz,
           (long long)nn);
    return ok ? 0 : 3;
}
"""


def _fmt(a):
    return ", ".join(repr(float(v)) for v in np.asarray(a, dtype=np.float64).ravel())


@pytest.mark.skipif(shutil.which("gcc") is None, reason="gcc not found")
def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    w = W.cube(6, 0.1, seed=7, correction=1.0, eps_s=0.2, n_s=4.0, xsph=0.5, eos=2.0,
               alpha=1.0, beta=1.0)
    rng = np.random.default_rng(7)
    n = w.n
    u = rng.uniform(0.0, 2e7, n)
    d = rng.uniform(0.0, 1.0, n)
    w.rho = w.params["rho0"] * rng.uniform(0.97, 1.03, n)
    src = (DRIVER.replace("POS_VALUES", _fmt(w.pos)).replace("VEL_VALUES", _fmt(w.vel))
           .replace("RHO_VALUES", _fmt(w.rho)).replace("S_VALUES", _fmt(w.S))
           .replace("M_VALUES", _fmt(w.m)).replace("U_VALUES", _fmt(u))
           .replace("D_VALUES", _fmt(d)).replace("PAR_VALUES", _fmt(w.param_vector()))
           .replace("NUM", str(n)))
    drv = tmp_path / "driver.c"
    drv.write_text(src)
    exe = tmp_path / "driver"
    cmd = ["gcc", "-O1", "-g", "-std=c99", "-fno-omit-frame-pointer", "-ffp-contract=off",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-Wno-unknown-pragmas",
           str(drv), os.path.join(ORACLE, "sph_oracle.c"), os.path.join(ORACLE, "gravity.c"),
           "-o", str(exe), "-lm"]
    subprocess.run(cmd, check=True, capture_output=True, text=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:verify_asan_link_order=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "driver ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
