"""The C oracles under AddressSanitizer and UndefinedBehaviorSanitizer.

A small C driver calls the MCLAHE oracle (every dimensionality 1..4, every
dtype, both range modes, a caller range, every redistribution variant, both
centre conventions, integer output) and the Gaussian oracle on tiny inputs,
built with -fsanitize=address,undefined (gcc, host code only).  Any report or
a non-zero exit fails the test.
"""
import os
import shutil
import subprocess
import tempfile

import pytest

import oracle

HERE = os.path.dirname(oracle.__file__)

DRIVER = r"""
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
int mclahe_oracle_run_variant(int, const int64_t *, const int64_t *, int, float, int, const float *, int,
                              const void *, int, void *, int64_t *, int64_t *, float *, float *, double *,
                              int, int, int);
int denoise_oracle_gaussian(int, const int64_t *, int, const void *, const double *, double, float *);
static unsigned lcg(unsigned *s) { *s = *s * 1664525u + 1013904223u; return *s >> 8; }
int main(void)
{
    unsigned seed = 7;
    const int64_t shapes[4][4] = {{13, 0, 0, 0}, {9, 7, 0, 0}, {6, 5, 4, 0}, {5, 4, 3, 3}};
    const int64_t kss[4][4] = {{4, 0, 0, 0}, {3, 7, 0, 0}, {2, 5, 1, 0}, {5, 2, 3, 1}};
    int runs = 0;
    for (int D = 1; D <= 4; ++D) {
        int64_t n = 1, nk_max = 1;
        for (int i = 0; i < D; ++i) { n *= shapes[D - 1][i]; nk_max *= shapes[D - 1][i] + 2; }
        float *xf = malloc(sizeof(float) * n);
        uint16_t *xu = malloc(sizeof(uint16_t) * n);
        uint8_t *xb = malloc(n);
        for (int64_t i = 0; i < n; ++i) {
            const unsigned r = lcg(&seed) % 40;
            xf[i] = (float)r * 0.37f; xu[i] = (uint16_t)(r * 900); xb[i] = (uint8_t)(r * 6);
        }
        const int nb = 8;
        float *outf = malloc(sizeof(float) * n);
        int64_t *hist = malloc(sizeof(int64_t) * nk_max * nb), *cl = malloc(sizeof(int64_t) * nk_max * nb);
        float *lut = malloc(sizeof(float) * nk_max * nb), *rng = malloc(sizeof(float) * 2 * nk_max);
        double *f64 = malloc(sizeof(double) * n);
        const void *ins[3] = {xb, xu, xf};
        for (int dt = 0; dt < 3; ++dt)
            for (int mode = 0; mode < 2; ++mode)
                for (int red = 0; red < 3; ++red)
                    for (int ch = 0; ch < 2; ++ch)
                        for (int od = 0; od < 3; od += 2) {
                            const float ur[2] = {0.f, 20.f};
                            const int rc = mclahe_oracle_run_variant(D, shapes[D - 1], kss[D - 1], nb, 0.2f, mode,
                                                                     (mode == 0 && red == 1) ? ur : NULL, dt, ins[dt],
                                                                     od, outf, hist, cl, lut, rng, f64, red, 3, ch);
                            if (rc) { printf("run failed rc=%d\n", rc); return 2; }
                            ++runs;
                        }
        const double sig[4] = {0.7, 1.3, 0.0, 0.9};
        if (denoise_oracle_gaussian(D, shapes[D - 1], 2, xf, sig, 4.0, outf)) { printf("gauss failed\n"); return 3; }
        free(xf); free(xu); free(xb); free(outf); free(hist); free(cl); free(lut); free(rng); free(f64);
    }
    printf("ok %d runs\n", runs);
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
def test_oracles_clean_under_asan_ubsan():
    d = tempfile.mkdtemp(prefix="oracle_san_")
    drv = os.path.join(d, "drv.c")
    exe = os.path.join(d, "drv")
    open(drv, "w").write(DRIVER)
    cmd = ["gcc", "-O1", "-g", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fno-omit-frame-pointer",
           "-fsanitize=address,undefined", "-fno-sanitize-recover=undefined",
           drv, os.path.join(HERE, "mclahe_oracle.c"), os.path.join(HERE, "denoise_oracle.c"), "-o", exe, "-lm"]
    subprocess.check_call(cmd)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1", OMP_NUM_THREADS="2")
    r = subprocess.run([exe], capture_output=True, text=True, env=env, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
    assert r.stdout.startswith("ok ")
