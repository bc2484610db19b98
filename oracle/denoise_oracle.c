/*
 * Pre-denoising filter of the paper's experiments -- TEST INFRASTRUCTURE ONLY.
 *
 * Before CLAHE, the photoemission volume of Sec. IV.A is smoothed with a
 * Gaussian filter of a given standard deviation per axis.  The paper gives
 * the deviations and nothing else; this oracle states the reading the GPU
 * library implements, as plain loops.  Only the tests, the smoke check and
 * the benchmark's CPU leg may load it; it shares no code with the library.
 *
 * Readings:
 *  - the filter is separable: one 1-D pass per axis, axes in order 0..D-1,
 *    axes with sigma <= 0 left alone;
 *  - the 1-D kernel has radius r = (int)(truncate * sigma + 0.5) (truncate
 *    = 4 by default) and weights phi_j = exp(-0.5 / (sigma * sigma) * j^2),
 *    j = -r..r, divided by their sum (both in double, summed in order of j)
 *    and rounded to float;
 *  - outside the array the data continue by edge-repeating reflection, the
 *    padding of the CLAHE method itself ([a b c] -> [.. b a | a b c | c b ..],
 *    period 2n, any radius);
 *  - every pass works in single precision: out_p = w_{-r} x_{p-r} + ... +
 *    w_r x_{p+r}, accumulated in order of j with a fused multiply-add per
 *    term starting from 0, and stored as float (so that both sides take the
 *    same integer decisions when the result is binned);
 *  - input u8, u16 or float (converted exactly to float); output float.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

enum { DN_U8 = 0, DN_U16 = 1, DN_F32 = 2 };
#define DN_MAX_DIM 8
#define DN_MAX_RADIUS 64

/* Index i (any integer) of a line of n samples under edge-repeating reflection. */
static int64_t reflect_index(int64_t i, int64_t n)
{
    const int64_t period = 2 * n;
    i %= period;
    if (i < 0) i += period;
    return i < n ? i : period - 1 - i;
}

int denoise_oracle_gauss_radius(double sigma, double truncate)
{
    if (!(sigma > 0.0) || !(truncate > 0.0)) return 0;
    return (int)(truncate * sigma + 0.5);
}

/* Weights w[0..2r] of the kernel; returns r, or -1 if r is too large. */
int denoise_oracle_gauss_weights(double sigma, double truncate, float *w)
{
    const int r = denoise_oracle_gauss_radius(sigma, truncate);
    if (r > DN_MAX_RADIUS) return -1;
    double phi[2 * DN_MAX_RADIUS + 1], sum = 0.0;
    for (int j = -r; j <= r; ++j) {
        phi[j + r] = exp(-0.5 / (sigma * sigma) * (double)(j * j));
        sum += phi[j + r];
    }
    for (int j = 0; j <= 2 * r; ++j) w[j] = (float)(phi[j] / sum);
    return r;
}

/* One term of the accumulation: correctly rounded single-precision fused
 * multiply-add (in hardware where the CPU has it, else in libm; the value
 * is the same). */
__attribute__((target("fma"))) static void pass_fma(const float *a, float *b, int64_t nvox, int64_t S,
                                                    int64_t n, int r, const float *w)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nvox; ++e) {
        const int64_t p = (e / S) % n, base = e - p * S;
        float acc = 0.0f;
        for (int j = -r; j <= r; ++j) acc = __builtin_fmaf(w[j + r], a[base + reflect_index(p + j, n) * S], acc);
        b[e] = acc;
    }
}

static void pass_libm(const float *a, float *b, int64_t nvox, int64_t S, int64_t n, int r, const float *w)
{
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < nvox; ++e) {
        const int64_t p = (e / S) % n, base = e - p * S;
        float acc = 0.0f;
        for (int j = -r; j <= r; ++j) acc = fmaf(w[j + r], a[base + reflect_index(p + j, n) * S], acc);
        b[e] = acc;
    }
}

/* Gaussian smoothing of a C-contiguous array; returns 0, 1 (bad argument)
 * or 2 (allocation failed). */
int denoise_oracle_gaussian(int D, const int64_t *shape, int in_dtype, const void *in, const double *sigma,
                            double truncate, float *out)
{
    if (D < 1 || D > DN_MAX_DIM || !shape || !in || !sigma || !out) return 1;
    int64_t nvox = 1;
    for (int i = 0; i < D; ++i) {
        if (shape[i] < 1) return 1;
        nvox *= shape[i];
    }
    float *a = malloc(sizeof(float) * nvox), *b = malloc(sizeof(float) * nvox);
    if (!a || !b) {
        free(a);
        free(b);
        return 2;
    }
    for (int64_t e = 0; e < nvox; ++e)
        a[e] = in_dtype == DN_U8 ? (float)((const uint8_t *)in)[e]
             : in_dtype == DN_U16 ? (float)((const uint16_t *)in)[e] : ((const float *)in)[e];
    const int use_fma = __builtin_cpu_supports("fma");
    int64_t S = nvox;
    for (int ax = 0; ax < D; ++ax) {
        S /= shape[ax];                       /* stride of axis ax */
        if (!(sigma[ax] > 0.0)) continue;
        float w[2 * DN_MAX_RADIUS + 1];
        const int r = denoise_oracle_gauss_weights(sigma[ax], truncate, w);
        if (r < 0) {
            free(a);
            free(b);
            return 1;
        }
        if (use_fma) pass_fma(a, b, nvox, S, shape[ax], r, w);
        else pass_libm(a, b, nvox, S, shape[ax], r, w);
        float *t = a;
        a = b;
        b = t;
    }
    memcpy(out, a, sizeof(float) * nvox);
    free(a);
    free(b);
    return 0;
}
