// Pre-denoising filters applied before CLAHE in the paper's experiments
// (Sec. IV): a separable Gaussian with a standard deviation per axis
// (photoemission volume) and a median filter over a small window
// (fluorescence microscopy volume, window (2, 2, 2, 1)).
//
// Gaussian: one pass per axis with sigma > 0, axes in order; radius
// r = (int)(truncate * sigma + 0.5); weights exp(-0.5 / sigma^2 * j^2) over
// their sum, in double on the host, rounded to float; edge-repeating
// reflection outside the array (the CLAHE padding, period 2n); every output
// is the float32 fused multiply-add chain over j = -r..r starting from 0, so
// the result is bit-identical to a plain loop that does the same.
//   - last axis (contiguous): a work-group stages a flat tile of 2048 outputs
//     plus r halo samples on each side in LDS (reflection never reaches
//     further than r from an output) and every thread filters 8 outputs;
//   - any other axis (stride S): a thread owns 4 (or 1) adjacent columns and
//     sweeps a segment of the axis with a ring of 2r + 1 samples in
//     registers, unrolled by the ring length so that every slot index is a
//     compile-time constant: each input is loaded once per segment.
// Median: one output per thread; the window's values are gathered with
// reflected coordinates and sorted by a bitonic network padded to a power
// of two; the value of rank N / 2 (0-based) is written in the input dtype.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <vector>

#include "../../include/mclahe.h"
#include "mc_launch.h"

namespace {

constexpr int kT = 256;
constexpr int kTile = 2048;          // outputs per work-group on the last axis
constexpr int kRingMax = 8;          // largest radius with a register ring
constexpr int kRadiusMax = 64;       // largest radius at all
constexpr int kMedianMax = 64;       // largest median window (values)

struct Weights {
    float w[2 * kRadiusMax + 1];
};

__device__ __forceinline__ int64_t refl(int64_t i, int64_t n)
{
    if (i >= 0 && i < n) return i;
    const int64_t period = 2 * n;
    i %= period;
    if (i < 0) i += period;
    return i < n ? i : period - 1 - i;
}

template <typename T>
__device__ __forceinline__ float ld1(const T *p, int64_t i)
{
    return (float)p[i];
}

// ------------------------------------------------------------- last axis --
template <typename T>
__global__ void __launch_bounds__(kT) k_gauss_last(const T *in, float *out, int64_t nvox, int64_t n, int r,
                                                  Weights W)
{
    extern __shared__ float tile[];   // [kTile + 2r]
    const int64_t e0 = (int64_t)blockIdx.x * kTile;
    const int64_t lo = e0 - r;
    const int len = kTile + 2 * r;
    for (int i = threadIdx.x; i < len; i += kT) {
        const int64_t e = lo + i;
        tile[i] = (e >= 0 && e < nvox) ? ld1(in, e) : 0.f;
    }
    __syncthreads();
#pragma unroll 2
    for (int k = 0; k < kTile / kT; ++k) {
        const int t = threadIdx.x + k * kT;
        const int64_t e = e0 + t;
        if (e >= nvox) break;
        const int64_t p = e % n;
        float acc = 0.f;
        if (p >= r && p + r < n) {
            for (int j = -r; j <= r; ++j) acc = __builtin_fmaf(W.w[j + r], tile[t + r + j], acc);
        } else {
            for (int j = -r; j <= r; ++j) {
                const int64_t q = e - p + refl(p + j, n);   // same row, within r of e
                acc = __builtin_fmaf(W.w[j + r], tile[(int)(q - lo)], acc);
            }
        }
        out[e] = acc;
    }
}

// ---------------------------------------------------------- strided axes --
template <int V> struct VecF;
template <> struct VecF<1> { float v[1]; };
template <> struct VecF<4> { float v[4]; };

template <typename T, int V>
__device__ __forceinline__ VecF<V> ldv(const T *p, int64_t i)
{
    VecF<V> r;
    if constexpr (V == 4 && sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(p + i);
        r.v[0] = a.x; r.v[1] = a.y; r.v[2] = a.z; r.v[3] = a.w;
    } else if constexpr (V == 4 && sizeof(T) == 2) {
        const uint2 a = *reinterpret_cast<const uint2 *>(p + i);
        r.v[0] = (float)(a.x & 0xffffu); r.v[1] = (float)(a.x >> 16);
        r.v[2] = (float)(a.y & 0xffffu); r.v[3] = (float)(a.y >> 16);
    } else if constexpr (V == 4 && sizeof(T) == 1) {
        const uint32_t a = *reinterpret_cast<const uint32_t *>(p + i);
#pragma unroll
        for (int k = 0; k < 4; ++k) r.v[k] = (float)((a >> (8 * k)) & 0xffu);
    } else {
#pragma unroll
        for (int k = 0; k < V; ++k) r.v[k] = (float)p[i + k];
    }
    return r;
}

template <int V>
__device__ __forceinline__ void stv(float *p, int64_t i, const float (&a)[V])
{
    if constexpr (V == 4) *reinterpret_cast<float4 *>(p + i) = make_float4(a[0], a[1], a[2], a[3]);
    else p[i] = a[0];
}

// Column geometry of a strided pass: the array is [outer][n][S]; a "column"
// is one (outer, s) pair, V adjacent s per thread.
struct Cols {
    int64_t n, S, vcols;   // axis length, stride, vector columns = outer * S / V
    int64_t seg, nseg;     // positions per segment, segments per column
};

template <typename T, int V, int R>
__global__ void __launch_bounds__(kT) k_gauss_ring(const T *in, float *out, Cols c, Weights W)
{
    constexpr int WN = 2 * R + 1;
    const int64_t gid = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t col = gid % c.vcols, sg = gid / c.vcols;
    if (sg >= c.nseg) return;
    const int64_t s0 = (col * V) % c.S, outer = (col * V) / c.S;
    const int64_t base = outer * c.n * c.S + s0;
    const int64_t p0 = sg * c.seg, p1 = std::min(p0 + c.seg, c.n);
    float w[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j) w[j] = W.w[j];
    VecF<V> ring[WN];
    // slot of input position q: (q - (p0 - R)) mod WN
#pragma unroll
    for (int j = 0; j < 2 * R; ++j) ring[j] = ldv<T, V>(in, base + refl(p0 - R + j, c.n) * c.S);
    for (int64_t pb = p0; pb < p1; pb += WN) {
#pragma unroll
        for (int u = 0; u < WN; ++u) {
            const int64_t p = pb + u;
            if (p < p1) {
                ring[(u + 2 * R) % WN] = ldv<T, V>(in, base + refl(p + R, c.n) * c.S);
                float acc[V];
#pragma unroll
                for (int k = 0; k < V; ++k) acc[k] = 0.f;
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int k = 0; k < V; ++k) acc[k] = __builtin_fmaf(w[j], ring[(u + j) % WN].v[k], acc[k]);
                stv<V>(out, base + p * c.S, acc);
            }
        }
    }
}

// Any radius: the taps are loaded directly (caches serve the reuse).
template <typename T, int V>
__global__ void __launch_bounds__(kT) k_gauss_direct(const T *in, float *out, Cols c, int r, Weights W)
{
    const int64_t gid = (int64_t)blockIdx.x * kT + threadIdx.x;
    const int64_t col = gid % c.vcols, sg = gid / c.vcols;
    if (sg >= c.nseg) return;
    const int64_t s0 = (col * V) % c.S, outer = (col * V) / c.S;
    const int64_t base = outer * c.n * c.S + s0;
    const int64_t p0 = sg * c.seg, p1 = std::min(p0 + c.seg, c.n);
    for (int64_t p = p0; p < p1; ++p) {
        float acc[V];
#pragma unroll
        for (int k = 0; k < V; ++k) acc[k] = 0.f;
        for (int j = -r; j <= r; ++j) {
            const VecF<V> x = ldv<T, V>(in, base + refl(p + j, c.n) * c.S);
#pragma unroll
            for (int k = 0; k < V; ++k) acc[k] = __builtin_fmaf(W.w[j + r], x.v[k], acc[k]);
        }
        stv<V>(out, base + p * c.S, acc);
    }
}

// Plain conversion to float (no axis to smooth).
template <typename T>
__global__ void __launch_bounds__(kT) k_to_float(const T *in, float *out, int64_t nvox)
{
    for (int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x; e < nvox; e += (int64_t)gridDim.x * kT)
        out[e] = (float)in[e];
}

// ----------------------------------------------------------------- median --
struct MedGeom {
    int D, N;                        // dims, window values
    int64_t shape[MC_MAXD], stride[MC_MAXD];
    int32_t lo[MC_MAXD], k[MC_MAXD]; // window offsets lo .. lo + k - 1 per axis
    int64_t nvox;
};

template <int NP>
__device__ __forceinline__ void bitonic_sort(float (&a)[NP])
{
#pragma unroll
    for (int size = 2; size <= NP; size <<= 1)
#pragma unroll
        for (int stride = size >> 1; stride > 0; stride >>= 1)
#pragma unroll
            for (int i = 0; i < NP; ++i) {
                const int j = i ^ stride;
                if (j > i) {
                    const bool up = (i & size) == 0;
                    const float x = a[i], y = a[j];
                    a[i] = up ? fminf(x, y) : fmaxf(x, y);
                    a[j] = up ? fmaxf(x, y) : fminf(x, y);
                }
            }
}

template <typename T, int NP>
__global__ void __launch_bounds__(kT) k_median(const T *in, T *out, MedGeom g)
{
    const int64_t e = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (e >= g.nvox) return;
    int64_t pos[MC_MAXD];
    int64_t rem = e;
    for (int a = 0; a < g.D; ++a) {
        pos[a] = rem / g.stride[a];
        rem -= pos[a] * g.stride[a];
    }
    float v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        v[i] = INFINITY;   // padding sorts last: the rank below N is unchanged
        if (i < g.N) {
            int q = i;
            int64_t off = 0;
            for (int a = g.D - 1; a >= 0; --a) {
                const int o = q % g.k[a];
                q /= g.k[a];
                off += refl(pos[a] + g.lo[a] + o, g.shape[a]) * g.stride[a];
            }
            v[i] = (float)in[off];
        }
    }
    bitonic_sort<NP>(v);
    float m = v[0];
#pragma unroll
    for (int i = 0; i < NP; ++i)
        if (i == g.N / 2) m = v[i];
    out[e] = (T)m;
}

// ------------------------------------------------------------------ host --
int gauss_radius(double sigma, double truncate)
{
    return sigma > 0.0 ? (int)(truncate * sigma + 0.5) : 0;
}

void gauss_weights(double sigma, double truncate, Weights &W, int &r)
{
    r = gauss_radius(sigma, truncate);
    double phi[2 * kRadiusMax + 1], sum = 0.0;
    for (int j = -r; j <= r; ++j) {
        phi[j + r] = std::exp(-0.5 / (sigma * sigma) * (double)(j * j));
        sum += phi[j + r];
    }
    for (int j = 0; j < 2 * kRadiusMax + 1; ++j) W.w[j] = j <= 2 * r ? (float)(phi[j] / sum) : 0.f;
}

mclahe_status check_shape(int ndim, const int64_t *shape, int64_t &nvox)
{
    if (ndim < 1 || ndim > MC_MAXD || !shape)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "ndim must be in [1, %d]", MC_MAXD);
    nvox = 1;
    for (int i = 0; i < ndim; ++i) {
        if (shape[i] < 1) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "shape[%d] must be >= 1", i);
        nvox *= shape[i];
    }
    return MCLAHE_SUCCESS;
}

template <typename T>
mclahe_status gauss_pass(const T *in, float *out, int64_t nvox, int64_t n, int64_t S, int r, const Weights &W,
                         hipStream_t st)
{
    if (S == 1) {
        const int64_t blocks = (nvox + kTile - 1) / kTile;
        hipLaunchKernelGGL(k_gauss_last<T>, dim3((uint32_t)blocks), dim3(kT), sizeof(float) * (kTile + 2 * r), st,
                           in, out, nvox, n, r, W);
    } else {
        const bool vec = S % 4 == 0 && ((uintptr_t)in % (4 * sizeof(T))) == 0 && ((uintptr_t)out % 16) == 0;
        const int V = vec ? 4 : 1;
        Cols c;
        c.n = n;
        c.S = S;
        c.vcols = nvox / n / V;
        // segments: a multiple of the ring length near 64 positions, fewer
        // if the columns alone do not fill the chip
        const int WN = 2 * r + 1;
        int64_t seg = ((64 + WN - 1) / WN) * WN;
        const int64_t want_threads = 256LL * 2048;
        while (seg > WN && c.vcols * ((n + seg - 1) / seg) < want_threads) seg -= WN;
        c.seg = std::min<int64_t>(seg, n);
        c.nseg = (n + c.seg - 1) / c.seg;
        const int64_t blocks = (c.vcols * c.nseg + kT - 1) / kT;
        if (blocks > 0x7fffffff) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large for one pass");
        const dim3 grid((uint32_t)blocks), blk(kT);
#define RING(RR)                                                                              \
    case RR:                                                                                  \
        if (vec) hipLaunchKernelGGL((k_gauss_ring<T, 4, RR>), grid, blk, 0, st, in, out, c, W); \
        else hipLaunchKernelGGL((k_gauss_ring<T, 1, RR>), grid, blk, 0, st, in, out, c, W);     \
        break;
        switch (r) {
            RING(1) RING(2) RING(3) RING(4) RING(5) RING(6) RING(7) RING(8)
        default:
            if (vec) hipLaunchKernelGGL((k_gauss_direct<T, 4>), grid, blk, 0, st, in, out, c, r, W);
            else hipLaunchKernelGGL((k_gauss_direct<T, 1>), grid, blk, 0, st, in, out, c, r, W);
        }
#undef RING
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "gaussian pass launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

template <typename T>
mclahe_status median_launch(const void *in, void *out, const MedGeom &g, hipStream_t st)
{
    const uint32_t blocks = (uint32_t)((g.nvox + kT - 1) / kT);
    const T *i = (const T *)in;
    T *o = (T *)out;
    if (g.N <= 2) hipLaunchKernelGGL((k_median<T, 2>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    else if (g.N <= 4) hipLaunchKernelGGL((k_median<T, 4>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    else if (g.N <= 8) hipLaunchKernelGGL((k_median<T, 8>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    else if (g.N <= 16) hipLaunchKernelGGL((k_median<T, 16>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    else if (g.N <= 32) hipLaunchKernelGGL((k_median<T, 32>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    else hipLaunchKernelGGL((k_median<T, 64>), dim3(blocks), dim3(kT), 0, st, i, o, g);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "median launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

}  // namespace

extern "C" {

mclahe_status mclahe_gaussian_workspace_size(int ndim, const int64_t *shape, const double *sigma, size_t *bytes)
{
    mc_clear_error();
    int64_t nvox;
    mclahe_status s = check_shape(ndim, shape, nvox);
    if (s) return s;
    if (!sigma || !bytes) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "sigma and bytes must not be NULL");
    int passes = 0;
    for (int i = 0; i < ndim; ++i) passes += sigma[i] > 0.0;
    *bytes = passes >= 2 ? ((sizeof(float) * nvox + 255) & ~size_t(255)) : 0;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_gaussian(const void *d_in, mclahe_dtype in_dtype, int ndim, const int64_t *shape,
                              const double *sigma, double truncate, float *d_out, void *d_workspace,
                              size_t workspace_bytes, void *hip_stream)
{
    size_t need = 0;
    mclahe_status s = mclahe_gaussian_workspace_size(ndim, shape, sigma, &need);
    if (s) return s;
    if (!d_in || !d_out) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "input and output must not be NULL");
    if (in_dtype != MCLAHE_U8 && in_dtype != MCLAHE_U16 && in_dtype != MCLAHE_F32)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "unknown dtype");
    if (!(truncate > 0.0) || !std::isfinite(truncate))
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "truncate must be positive and finite");
    for (int i = 0; i < ndim; ++i) {
        if (!(sigma[i] >= 0.0) || !std::isfinite(sigma[i]))
            return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "sigma[%d] must be finite and >= 0", i);
        if (gauss_radius(sigma[i], truncate) > kRadiusMax)
            return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "sigma[%d] gives a radius over %d", i, kRadiusMax);
    }
    int64_t nvox = 1;
    for (int i = 0; i < ndim; ++i) nvox *= shape[i];
    const size_t esz = in_dtype == MCLAHE_U8 ? 1 : in_dtype == MCLAHE_U16 ? 2 : 4;
    const char *ib = (const char *)d_in, *ob = (const char *)d_out;
    if (ib < ob + sizeof(float) * nvox && ob < ib + esz * nvox)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "input and output must not overlap");
    if (need && (!d_workspace || ((uintptr_t)d_workspace & 255) || workspace_bytes < need))
        return mc_fail(MCLAHE_ERROR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned", need);
    hipStream_t st = (hipStream_t)hip_stream;
    std::vector<int> axes;
    for (int i = 0; i < ndim; ++i)
        if (sigma[i] > 0.0) axes.push_back(i);
    const int P = (int)axes.size();
    if (P == 0) {
        const uint32_t blocks = (uint32_t)std::min<int64_t>(4096, (nvox + kT - 1) / kT);
        if (in_dtype == MCLAHE_U8) hipLaunchKernelGGL(k_to_float<uint8_t>, dim3(blocks), dim3(kT), 0, st, (const uint8_t *)d_in, d_out, nvox);
        else if (in_dtype == MCLAHE_U16) hipLaunchKernelGGL(k_to_float<uint16_t>, dim3(blocks), dim3(kT), 0, st, (const uint16_t *)d_in, d_out, nvox);
        else hipLaunchKernelGGL(k_to_float<float>, dim3(blocks), dim3(kT), 0, st, (const float *)d_in, d_out, nvox);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? MCLAHE_SUCCESS : mc_fail(MCLAHE_ERROR_HIP, "launch failed: %s", hipGetErrorString(e));
    }
    float *tmp = (float *)d_workspace;
    const float *src = nullptr;
    for (int k = 0; k < P; ++k) {
        const int a = axes[k];
        int64_t S = 1;
        for (int i = a + 1; i < ndim; ++i) S *= shape[i];
        Weights W;
        int r;
        gauss_weights(sigma[a], truncate, W, r);
        float *dst = ((P - 1 - k) % 2 == 0) ? d_out : tmp;   // the last pass lands in d_out
        if (k == 0) {
            if (in_dtype == MCLAHE_U8) s = gauss_pass<uint8_t>((const uint8_t *)d_in, dst, nvox, shape[a], S, r, W, st);
            else if (in_dtype == MCLAHE_U16) s = gauss_pass<uint16_t>((const uint16_t *)d_in, dst, nvox, shape[a], S, r, W, st);
            else s = gauss_pass<float>((const float *)d_in, dst, nvox, shape[a], S, r, W, st);
        } else {
            s = gauss_pass<float>(src, dst, nvox, shape[a], S, r, W, st);
        }
        if (s) return s;
        src = dst;
    }
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_median(const void *d_in, mclahe_dtype dtype, int ndim, const int64_t *shape,
                            const int32_t *window, void *d_out, void *hip_stream)
{
    mc_clear_error();
    int64_t nvox;
    mclahe_status s = check_shape(ndim, shape, nvox);
    if (s) return s;
    if (!d_in || !d_out || !window) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (dtype != MCLAHE_U8 && dtype != MCLAHE_U16 && dtype != MCLAHE_F32)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "unknown dtype");
    MedGeom g{};
    g.D = ndim;
    g.nvox = nvox;
    int64_t N = 1;
    for (int i = 0; i < ndim; ++i) {
        if (window[i] < 1) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "window[%d] must be >= 1", i);
        N *= window[i];
        if (N > kMedianMax) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "window over %d values", kMedianMax);
        g.shape[i] = shape[i];
        g.k[i] = window[i];
        g.lo[i] = -(window[i] / 2);
    }
    g.N = (int)N;
    int64_t st = 1;
    for (int i = ndim - 1; i >= 0; --i) {
        g.stride[i] = st;
        st *= shape[i];
    }
    const size_t esz = dtype == MCLAHE_U8 ? 1 : dtype == MCLAHE_U16 ? 2 : 4;
    const char *ib = (const char *)d_in, *ob = (const char *)d_out;
    if (ib < ob + esz * nvox && ob < ib + esz * nvox)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "input and output must not overlap");
    if ((nvox + kT - 1) / kT > 0x7fffffff) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large");
    hipStream_t hs = (hipStream_t)hip_stream;
    if (dtype == MCLAHE_U8) return median_launch<uint8_t>(d_in, d_out, g, hs);
    if (dtype == MCLAHE_U16) return median_launch<uint16_t>(d_in, d_out, g, hs);
    return median_launch<float>(d_in, d_out, g, hs);
}

}  // extern "C"
