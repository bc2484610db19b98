/*
 * Plain CPU oracle for multidimensional CLAHE (MCLAHE, Stimper et al., 2019).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * statement of what the GPU library computes.  Only the test-suite, the smoke
 * check and the CPU-baseline leg of the benchmark may load it.  It shares no
 * code, header, table or constant with the HIP library and includes nothing
 * from it.
 *
 * It follows the paper's Algorithm 1 step by step:
 *   1. padding length per axis                       (Sec. III.B, Eq. 1)
 *   2. symmetric padding, split p//2 and (p+1)//2     (Sec. III.B, Eq. 2)
 *   3. split the padded data into kernels             (Sec. III.A overview)
 *   4. per-kernel histogram with n_bins bins          (Alg. 1, histogram step)
 *   5. clip at clip_limit, redistribute equally       (Alg. 1, clip step)
 *   6. cumulative distribution                        (Alg. 1, cdf step)
 *   7. min-max normalised CDF as the mapping          (Alg. 1 map step; Sec. III.C)
 *   8. Lagrange multilinear interpolation over the 2^D nearest kernels
 *                                                      (Sec. III.C, coefficient product)
 * with the global (GHR) or adaptive, per-kernel (AHR) histogram range of
 * Sec. III.D.
 *
 * Readings of points the paper leaves open (all normative, identical on the
 * GPU side):
 *  - padding length uses the minus sign of Eq. 1 (the pseudo-code's plus sign
 *    would not make the padded size a multiple of the kernel size);
 *  - symmetric padding repeats the edge sample: [a b c] -> [b a | a b c | c b];
 *  - kernel_size[i] <= shape[i] is required;
 *  - GHR range is the data's min and max (or a caller-given range);
 *  - binning, in IEEE single precision without contraction:
 *        scale = (float)n / (hi - lo);  t = (v - lo) * scale;
 *        bin = t > 0 ? (t >= n ? n-1 : (int)t) : 0,  and if hi == lo:
 *        bin = v > lo ? n-1 : 0;
 *  - clip_limit is a fraction of the kernel's voxel count K: C = floor(clip*K),
 *    taken for the decimal the caller wrote: a double product that falls
 *    short of the next integer by no more than 2^-40 of itself is that
 *    integer (0.02 * 270000 -> 5400, 0.29 * 100 -> 29); C >= K clips nothing
 *    and is reported as K;
 *    the excess E = sum max(h-C, 0) is shared equally by all n bins, once.  In
 *    units of 1/n count that is exactly H_j = n*min(h_j, C) + E;
 *  - the CDF is inclusive; map_j = (cdf_j - cdf_0) / (cdf_{n-1} - cdf_0),
 *    evaluated in double and rounded to float; a zero denominator gives the
 *    ramp j/(n-1);
 *  - kernel centres sit at the middle of their voxel range, k*b + (b-1)/2 in
 *    padded coordinates; the interpolation weight towards the upper kernel is
 *    the distance to the lower centre over b;
 *  - the mapping of a voxel under a kernel is that kernel's map at the voxel's
 *    bin (computed with that kernel's range under AHR);
 *  - the 2^D contributions are summed (the pseudo-code's "assign" inside the
 *    neighbour loop is read as accumulate, as in the coefficient formula);
 *  - output is float in [0,1]; integer output is min(M, floor(y*M + 0.5))
 *    evaluated in single precision with M the dtype maximum.
 *
 * Variants for comparison with other CLAHE codes (mclahe_oracle_run_variant;
 * the defaults above are the paper's method):
 *  - repeated redistribution: after the equal share, bins above the clip
 *    level are clipped again and the new excess shared again, for at most
 *    `rounds` rounds, stopping early once no bin exceeds the level.  Round r
 *    works in integer units of 1/n^r count (the clip level becomes C*n^r);
 *  - integer redistribution: counts stay integers; every bin gets
 *    floor(E / n) and the remainder R = E mod n goes one count each to the
 *    bins 0, s, 2s, ... (R of them), s = max(n / R, 1);
 *  - kernel centres at k*b + b/2 (integer division) instead of k*b + (b-1)/2;
 *    the two coincide for odd b.
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -shared -fPIC (no fast-math).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_MAX_DIM 8

enum { ORC_U8 = 0, ORC_U16 = 1, ORC_F32 = 2 };
enum { ORC_GLOBAL = 0, ORC_KERNEL = 1 };
enum { ORC_REDIST_EQUAL = 0, ORC_REDIST_REPEATED = 1, ORC_REDIST_INTEGER = 2 };

/* Clip count of Algorithm 1's clip step: the clip limit is a fraction of the
 * kernel's K voxels.  The limit arrives as the binary double nearest the
 * decimal the caller wrote, so clip*K may land a rounding error below the
 * intended whole count; such a product is raised to that count. */
static int64_t oracle_clip_count(double clip_limit, int64_t K)
{
    const double c = clip_limit * (double)K;
    if (c >= (double)K) return K;                  /* no bin can exceed it */
    int64_t C = (int64_t)floor(c);
    if ((double)(C + 1) - c <= ldexp(c, -40)) C += 1;
    return C;
}

/* Eq. 1 and Eq. 2: padding per axis and its split; number of kernels. */
int mclahe_oracle_geometry(int ndim, const int64_t *shape, const int64_t *ksize,
                           int64_t *pad, int64_t *pad0, int64_t *pad1,
                           int64_t *nker)
{
    if (ndim < 1 || ndim > ORC_MAX_DIM) return 1;
    for (int i = 0; i < ndim; ++i) {
        int64_t s = shape[i], b = ksize[i];
        if (s < 1 || b < 1 || b > s) return 1;
        int64_t p = 2 * b - 1 - ((s - 1) % b);          /* Eq. 1 */
        pad[i] = p;
        pad0[i] = p / 2;                                 /* Eq. 2 */
        pad1[i] = (p + 1) / 2;
        nker[i] = (s + p) / b;   /* the padded size is a multiple of b */
    }
    return 0;
}

/* Symmetric (edge-repeating) mirror of a padded coordinate into [0, s). */
static int64_t mirror(int64_t q, int64_t p0, int64_t s)
{
    int64_t x = q - p0;
    if (x < 0) x = -x - 1;
    if (x >= s) x = 2 * s - 1 - x;
    return x;
}

/* Binning rule (reading of Alg. 1's histogram step), single precision. */
static int bin_of(float v, float lo, float hi, float scale, int n)
{
    if (hi == lo) return v > lo ? n - 1 : 0;
    float t = (v - lo) * scale;
    if (!(t > 0.0f)) return 0;
    if (t >= (float)n) return n - 1;
    return (int)t;
}

static float load_value(const void *in, int dtype, int64_t i)
{
    switch (dtype) {
    case ORC_U8: return (float)((const uint8_t *)in)[i];
    case ORC_U16: return (float)((const uint16_t *)in)[i];
    default: return ((const float *)in)[i];
    }
}

/*
 * Full MCLAHE.  Arrays are C-contiguous (last axis fastest).
 *   in        : input, dtype in_dtype, prod(shape) elements
 *   out       : output, dtype out_dtype (float in [0,1], or u8/u16 codes)
 *   hist      : [N_k][n_bins] int64 per-kernel histograms       (may be NULL)
 *   clipped   : [N_k][n_bins] int64 H = n*min(h,C) + E          (may be NULL)
 *   lut       : [N_k][n_bins] float maps                         (may be NULL)
 *   range     : [N_k][2] (AHR) or [2] (GHR) float lo, hi         (may be NULL)
 *   out_f64   : double interpolation result before rounding      (may be NULL)
 * Kernels are numbered row-major over the padded kernel grid.
 * Returns 0 on success, 1 on invalid arguments, 2 on allocation failure.
 */
int mclahe_oracle_run_variant(int ndim, const int64_t *shape, const int64_t *ksize,
                              int n_bins, double clip_limit, int mode,
                              const float *user_range, int in_dtype, const void *in,
                              int out_dtype, void *out, int64_t *hist, int64_t *clipped,
                              float *lut, float *range, double *out_f64,
                              int redistribution, int rounds, int centre_half)
{
    int64_t pad[ORC_MAX_DIM], pad0[ORC_MAX_DIM], pad1[ORC_MAX_DIM],
        nk[ORC_MAX_DIM];
    if (mclahe_oracle_geometry(ndim, shape, ksize, pad, pad0, pad1, nk)) return 1;
    if (n_bins < 2 || !(clip_limit >= 0.0) || isinf(clip_limit)) return 1;
    if (user_range && (mode != ORC_GLOBAL || !(user_range[0] < user_range[1]))) return 1;
    if (redistribution < ORC_REDIST_EQUAL || redistribution > ORC_REDIST_INTEGER || rounds < 1) return 1;
    const int D = ndim, n = n_bins;

    int64_t nvox = 1, npad = 1, nker = 1, K = 1;
    int64_t pshape[ORC_MAX_DIM];
    for (int i = 0; i < D; ++i) {
        pshape[i] = shape[i] + pad[i];
        nvox *= shape[i];
        npad *= pshape[i];
        nker *= nk[i];
        K *= ksize[i];
    }

    /* Alg. 1, padding step: materialise the symmetric padding. */
    float *padded = (float *)malloc((size_t)npad * sizeof(float));
    int64_t *h_all = (int64_t *)calloc((size_t)(nker * n), sizeof(int64_t));
    float *map = (float *)malloc((size_t)(nker * n) * sizeof(float));
    float *klo = (float *)malloc((size_t)nker * sizeof(float));
    float *khi = (float *)malloc((size_t)nker * sizeof(float));
    if (!padded || !h_all || !map || !klo || !khi) {
        free(padded); free(h_all); free(map); free(klo); free(khi);
        return 2;
    }
#pragma omp parallel for schedule(static)
    for (int64_t q = 0; q < npad; ++q) {
        int64_t rem = q, src = 0, stride = 1;
        int64_t qc[ORC_MAX_DIM];
        for (int i = D - 1; i >= 0; --i) { qc[i] = rem % pshape[i]; rem /= pshape[i]; }
        for (int i = D - 1; i >= 0; --i) {
            src += mirror(qc[i], pad0[i], shape[i]) * stride;
            stride *= shape[i];
        }
        padded[q] = load_value(in, in_dtype, src);
    }

    /* Sec. III.D: the histogram range, global or per kernel. */
    float glo = 0.0f, ghi = 0.0f;
    if (mode == ORC_GLOBAL) {
        if (user_range) {
            glo = user_range[0];
            ghi = user_range[1];
        } else {
            float mn = INFINITY, mx = -INFINITY;
#pragma omp parallel for reduction(min : mn) reduction(max : mx)
            for (int64_t i = 0; i < nvox; ++i) {
                float v = load_value(in, in_dtype, i);
                if (v < mn) mn = v;
                if (v > mx) mx = v;
            }
            glo = mn;
            ghi = mx;
        }
    }

    /* Alg. 1 loop over kernels: range (AHR), histogram, clip, cdf, map. */
    const int64_t C = oracle_clip_count(clip_limit, K);
#pragma omp parallel for schedule(dynamic)
    for (int64_t k = 0; k < nker; ++k) {
        int64_t kc[ORC_MAX_DIM], rem = k;
        for (int i = D - 1; i >= 0; --i) { kc[i] = rem % nk[i]; rem /= nk[i]; }
        /* enumerate the K padded voxels of kernel k */
        float lo = glo, hi = ghi;
        if (mode == ORC_KERNEL) {
            lo = INFINITY;
            hi = -INFINITY;
        }
        for (int pass = (mode == ORC_KERNEL ? 0 : 1); pass < 2; ++pass) {
            float scale = (float)n / (hi - lo);
            for (int64_t j = 0; j < K; ++j) {
                int64_t jr = j, off = 0, stride = 1;
                for (int i = D - 1; i >= 0; --i) {
                    int64_t qi = kc[i] * ksize[i] + jr % ksize[i];
                    jr /= ksize[i];
                    off += qi * stride;
                    stride *= pshape[i];
                }
                float v = padded[off];
                if (pass == 0) {
                    if (v < lo) lo = v;
                    if (v > hi) hi = v;
                } else {
                    h_all[k * n + bin_of(v, lo, hi, scale, n)] += 1;
                }
            }
        }
        klo[k] = lo;
        khi[k] = hi;

        int64_t *h = h_all + k * n;
        int64_t cdf0 = 0, cdfn = 0, acc = 0;
        int64_t *H = (int64_t *)malloc((size_t)n * sizeof(int64_t));
        if (redistribution == ORC_REDIST_INTEGER) {
            /* integer counts: an equal integer share, the remainder spread */
            int64_t E = 0;
            for (int j = 0; j < n; ++j) if (h[j] > C) E += h[j] - C;
            const int64_t q = E / n, R = E % n;
            const int64_t s = R ? (n / R > 1 ? n / R : 1) : 1;
            for (int j = 0; j < n; ++j)
                H[j] = (h[j] < C ? h[j] : C) + q + ((R && j % s == 0 && j / s < R) ? 1 : 0);
        } else {
            /* clip and redistribute the excess equally, in units of 1/n count;
             * repeated: again in units of 1/n^r while an excess remains */
            const int nr = redistribution == ORC_REDIST_REPEATED ? rounds : 1;
            int64_t Cr = C;
            for (int j = 0; j < n; ++j) H[j] = h[j];
            for (int r = 1; r <= nr; ++r) {
                int64_t E = 0;
                for (int j = 0; j < n; ++j) if (H[j] > Cr) E += H[j] - Cr;
                if (r > 1 && E == 0) break;
                for (int j = 0; j < n; ++j)
                    H[j] = (int64_t)n * (H[j] < Cr ? H[j] : Cr) + E;
                Cr *= n;
            }
        }
        for (int j = 0; j < n; ++j) {
            acc += H[j];                       /* inclusive cdf */
            if (j == 0) cdf0 = acc;
            if (clipped) clipped[k * n + j] = H[j];
        }
        cdfn = acc;
        acc = 0;
        for (int j = 0; j < n; ++j) {
            acc += H[j];
            double m = (cdfn == cdf0)
                           ? (double)j / (double)(n - 1)
                           : (double)(acc - cdf0) / (double)(cdfn - cdf0);
            map[k * n + j] = (float)m;
        }
        free(H);
    }

    /* Sec. III.C: multilinear interpolation over the 2^D nearest kernels. */
    const int ncorner = 1 << D;
    float gscale = (float)n / (ghi - glo);
#pragma omp parallel for schedule(static)
    for (int64_t x = 0; x < nvox; ++x) {
        int64_t xc[ORC_MAX_DIM], rem = x, k0[ORC_MAX_DIM];
        double w[ORC_MAX_DIM];
        for (int i = D - 1; i >= 0; --i) { xc[i] = rem % shape[i]; rem /= shape[i]; }
        for (int i = 0; i < D; ++i) {
            /* padded position minus the first kernel centre, doubled so that
             * it is an integer: m = 2*(x + p0) - (b - 1), or - 2*(b/2) with
             * the centre at b/2 */
            int64_t m = 2 * (xc[i] + pad0[i]) - (centre_half ? 2 * (ksize[i] / 2) : ksize[i] - 1);
            k0[i] = m / (2 * ksize[i]);
            w[i] = (double)(m - 2 * ksize[i] * k0[i]) / (double)(2 * ksize[i]);
        }
        float v = load_value(in, in_dtype, x);
        double y = 0.0;
        for (int c = 0; c < ncorner; ++c) {
            double coef = 1.0;
            int64_t kidx = 0;
            for (int i = 0; i < D; ++i) {
                int bit = (c >> (D - 1 - i)) & 1;
                coef *= bit ? w[i] : 1.0 - w[i];
                kidx = kidx * nk[i] + k0[i] + bit;
            }
            float lo = mode == ORC_KERNEL ? klo[kidx] : glo;
            float hi = mode == ORC_KERNEL ? khi[kidx] : ghi;
            float sc = mode == ORC_KERNEL ? (float)n / (hi - lo) : gscale;
            y += coef * (double)map[kidx * n + bin_of(v, lo, hi, sc, n)];
        }
        if (out_f64) out_f64[x] = y;
        float yf = (float)y;
        if (out_dtype == ORC_F32) {
            ((float *)out)[x] = yf;
        } else {
            float M = out_dtype == ORC_U8 ? 255.0f : 65535.0f;
            float qf = floorf(yf * M + 0.5f);
            if (qf > M) qf = M;
            if (qf < 0.0f) qf = 0.0f;
            if (out_dtype == ORC_U8) ((uint8_t *)out)[x] = (uint8_t)qf;
            else ((uint16_t *)out)[x] = (uint16_t)qf;
        }
    }

    if (hist) memcpy(hist, h_all, (size_t)(nker * n) * sizeof(int64_t));
    if (lut) memcpy(lut, map, (size_t)(nker * n) * sizeof(float));
    if (range) {
        if (mode == ORC_GLOBAL) {
            range[0] = glo;
            range[1] = ghi;
        } else {
            for (int64_t k = 0; k < nker; ++k) {
                range[2 * k] = klo[k];
                range[2 * k + 1] = khi[k];
            }
        }
    }
    free(padded); free(h_all); free(map); free(klo); free(khi);
    return 0;
}

/* The paper's method: equal redistribution once, centres at k*b + (b-1)/2. */
int mclahe_oracle_run(int ndim, const int64_t *shape, const int64_t *ksize,
                      int n_bins, double clip_limit, int mode,
                      const float *user_range, int in_dtype, const void *in,
                      int out_dtype, void *out, int64_t *hist, int64_t *clipped,
                      float *lut, float *range, double *out_f64)
{
    return mclahe_oracle_run_variant(ndim, shape, ksize, n_bins, clip_limit, mode, user_range, in_dtype, in,
                                     out_dtype, out, hist, clipped, lut, range, out_f64,
                                     ORC_REDIST_EQUAL, 1, 0);
}
