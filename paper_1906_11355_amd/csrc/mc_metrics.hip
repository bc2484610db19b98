// Contrast metrics on the GPU: mean squared error against an original, peak
// signal-to-noise ratio, RMS contrast (standard deviation) and grey-level
// Shannon entropy -- the four measures the paper judges enhancement by
// (Sec. II; Tables I and II).  Every volume is min-max normalised to [0, 1]
// before the metrics; the entropy histogram bins the raw values over the
// volume's own range with the CLAHE binning in single precision.
//
// Three stream-ordered passes over the data plus two one-work-group steps:
//   range : per work-group min, max and float64 sum of x (and y);
//   stats : lo, hi, normalised mean and binning scale of each volume; clears
//           the histogram counters;
//   accum : per voxel, float64 squared deviations from the normalised mean
//           and the squared difference of the two normalised volumes; LDS
//           grey-level histograms flushed into 64-bit counters.  Raw data
//           pile up on a few grey levels, and lanes of one wavefront adding
//           to one LDS word serialise: the lanes sharing the first lane's
//           bin add once, and every bin has R lane-interleaved copies
//           (lane l adds to copy l mod R) in consecutive words, i.e.
//           different banks;
//   final : reduces the partial sums in a fixed order and writes the result.
// The grid and the per-thread order are fixed, so results are reproducible
// bit for bit from run to run.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <type_traits>

#include "../../include/mclahe.h"
#include "mc_launch.h"

namespace {

constexpr int kT = 256;          // threads per work-group (4 wavefronts)
constexpr int kChunk = 8;        // elements per thread and step
constexpr int kMaxGroups = 2048; // 8 work-groups per compute unit
constexpr int kMaxBins = 8192;   // two LDS histograms of this many u32: 64 KiB
constexpr int kMaxCopies = 4;    // lane-interleaved copies of each bin
constexpr size_t kCopyLds = 32 * 1024;   // LDS the copies may take

// One per work-group of the range pass (or per interpolation unit of a
// CLAHE run that computes the metrics on the way): min, max, float64 sum.
using RangePart = McMetPart;
struct Stats {          // per volume, written by the stats step
    float lo[2], hi[2], scale[2];
    int32_t pad_;
    double inv[2];      // 1 / (hi - lo), 0 for a constant volume
    double off[2];      // -(lo * inv) - mean: fma(v, inv, off) = u - mean
    double dmean;       // mean_x - mean_y of the normalised volumes
    double mean[2];
};
struct AccPart {        // one per work-group of the accumulation pass
    double sxx, syy, sdd, pad_;
};

struct None {};          // "no second volume"

// Eight consecutive elements starting at element 8c, as floats (exact for
// u8 and u16).  VEC: one 8/16/32-byte access per thread (base aligned).
template <typename T, bool VEC>
__device__ __forceinline__ void load8(const T *p, int64_t c, float (&f)[kChunk])
{
    const T *q = p + c * kChunk;
    if constexpr (VEC && sizeof(T) == 4) {
        const float4 a = reinterpret_cast<const float4 *>(q)[0];
        const float4 b = reinterpret_cast<const float4 *>(q)[1];
        f[0] = a.x; f[1] = a.y; f[2] = a.z; f[3] = a.w;
        f[4] = b.x; f[5] = b.y; f[6] = b.z; f[7] = b.w;
    } else if constexpr (VEC && sizeof(T) == 2) {
        const uint4 a = reinterpret_cast<const uint4 *>(q)[0];
        const uint32_t w[4] = {a.x, a.y, a.z, a.w};
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            f[2 * k] = (float)(w[k] & 0xffffu);
            f[2 * k + 1] = (float)(w[k] >> 16);
        }
    } else if constexpr (VEC && sizeof(T) == 1) {
        const uint2 a = reinterpret_cast<const uint2 *>(q)[0];
        const uint32_t w[2] = {a.x, a.y};
#pragma unroll
        for (int k = 0; k < 8; ++k) f[k] = (float)((w[k >> 2] >> (8 * (k & 3))) & 0xffu);
    } else {
#pragma unroll
        for (int k = 0; k < kChunk; ++k) f[k] = (float)q[k];
    }
}

// Wavefront then work-group reductions (fixed order: the result does not
// depend on timing).
__device__ __forceinline__ double wave_sum(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}
__device__ __forceinline__ float wave_min(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fminf(v, __shfl_xor(v, o, 64));
    return v;
}
__device__ __forceinline__ float wave_max(float v)
{
    for (int o = 32; o > 0; o >>= 1) v = fmaxf(v, __shfl_xor(v, o, 64));
    return v;
}
// Sums of 4 wavefronts through LDS; every thread gets the total.
__device__ __forceinline__ double group_sum(double v, double *red)
{
    v = wave_sum(v);
    __syncthreads();
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
    __syncthreads();
    return (red[0] + red[1]) + (red[2] + red[3]);
}

// ---------------------------------------------------------------- range --
template <typename TX, typename TY, bool VEC>
__global__ void __launch_bounds__(kT) k_met_range(const TX *x, const TY *y, int64_t nvox, RangePart *part)
{
    constexpr bool HY = !std::is_same<TY, None>::value;
    __shared__ double red[4];
    __shared__ float redf[4][4];
    float mn[2] = {INFINITY, INFINITY}, mx[2] = {-INFINITY, -INFINITY};
    double s[2] = {0.0, 0.0};
    const int64_t nch = nvox / kChunk, stride = (int64_t)gridDim.x * kT;
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < nch; c += stride) {
        float fx[kChunk];
        load8<TX, VEC>(x, c, fx);
        float ts = 0.f;   // exact for integer data; float data sum in double below
        double ds = 0.0;
#pragma unroll
        for (int k = 0; k < kChunk; ++k) {
            mn[0] = fminf(mn[0], fx[k]);
            mx[0] = fmaxf(mx[0], fx[k]);
            if constexpr (sizeof(TX) < 4) ts += fx[k];
            else ds += (double)fx[k];
        }
        s[0] += sizeof(TX) < 4 ? (double)ts : ds;
        if constexpr (HY) {
            float fy[kChunk];
            load8<TY, VEC>(y, c, fy);
            float ty = 0.f;
            double dy = 0.0;
#pragma unroll
            for (int k = 0; k < kChunk; ++k) {
                mn[1] = fminf(mn[1], fy[k]);
                mx[1] = fmaxf(mx[1], fy[k]);
                if constexpr (sizeof(TY) < 4) ty += fy[k];
                else dy += (double)fy[k];
            }
            s[1] += sizeof(TY) < 4 ? (double)ty : dy;
        }
    }
    if (blockIdx.x == gridDim.x - 1) {   // elements past the last whole chunk
        for (int64_t t = nch * kChunk + threadIdx.x; t < nvox; t += kT) {
            const float a = (float)x[t];
            mn[0] = fminf(mn[0], a);
            mx[0] = fmaxf(mx[0], a);
            s[0] += (double)a;
            if constexpr (HY) {
                const float b = (float)y[t];
                mn[1] = fminf(mn[1], b);
                mx[1] = fmaxf(mx[1], b);
                s[1] += (double)b;
            }
        }
    }
    const int nv = HY ? 2 : 1;
    for (int v = 0; v < nv; ++v) {
        const float a = wave_min(mn[v]), b = wave_max(mx[v]);
        if ((threadIdx.x & 63) == 0) {
            redf[0][threadIdx.x >> 6] = a;
            redf[1][threadIdx.x >> 6] = b;
        }
        const double t = group_sum(s[v], red);   // its barriers publish redf too
        if (threadIdx.x == 0) {
            part[blockIdx.x].mn[v] = fminf(fminf(redf[0][0], redf[0][1]), fminf(redf[0][2], redf[0][3]));
            part[blockIdx.x].mx[v] = fmaxf(fmaxf(redf[1][0], redf[1][1]), fmaxf(redf[1][2], redf[1][3]));
            part[blockIdx.x].sum[v] = t;
        }
        __syncthreads();
    }
}

// ---------------------------------------------------------------- stats --
__global__ void __launch_bounds__(kT) k_met_stats(const RangePart *part, int groups, int nv, int64_t nvox,
                                                 int nb, Stats *st, unsigned long long *hist)
{
    __shared__ double red[4];
    __shared__ float redf[2][4];
    __shared__ double mean_s[2];
    for (int v = 0; v < nv; ++v) {
        float mn = INFINITY, mx = -INFINITY;
        double s = 0.0;
        for (int g = threadIdx.x; g < groups; g += kT) {
            mn = fminf(mn, part[g].mn[v]);
            mx = fmaxf(mx, part[g].mx[v]);
            s += part[g].sum[v];
        }
        mn = wave_min(mn);
        mx = wave_max(mx);
        if ((threadIdx.x & 63) == 0) {
            redf[0][threadIdx.x >> 6] = mn;
            redf[1][threadIdx.x >> 6] = mx;
        }
        const double tot = group_sum(s, red);
        if (threadIdx.x == 0) {
            const float lo = fminf(fminf(redf[0][0], redf[0][1]), fminf(redf[0][2], redf[0][3]));
            const float hi = fmaxf(fmaxf(redf[1][0], redf[1][1]), fmaxf(redf[1][2], redf[1][3]));
            const double inv = hi > lo ? 1.0 / ((double)hi - (double)lo) : 0.0;
            const double mean = (tot / (double)nvox - (double)lo) * inv;
            st->lo[v] = lo;
            st->hi[v] = hi;
            st->scale[v] = (float)nb / (hi - lo);   // +inf for a constant volume
            st->inv[v] = inv;
            st->off[v] = -((double)lo * inv) - mean;
            st->mean[v] = mean;
            mean_s[v] = mean;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) st->dmean = nv == 2 ? mean_s[0] - mean_s[1] : 0.0;
    for (int i = threadIdx.x; i < nv * nb; i += kT) hist[i] = 0ull;
}

// Bin of v in single precision, as the CLAHE histograms bin: t <= 0 and NaN
// give 0 (the saturating convert), t >= n gives n - 1.
__device__ __forceinline__ uint32_t met_bin(float v, float lo, float scale, uint32_t nbm1)
{
    const float t = (v - lo) * scale;
    return min(__float2uint_rz(t), nbm1);
}

// Count bin b of every active lane in copy (lane mod R) of an LDS histogram
// laid out [bin][R] (rs = log2 R): the lanes sharing the first active lane's
// bin add once, with their number; the others add one each.
__device__ __forceinline__ void count_bin(uint32_t *h, uint32_t b, int rs)
{
    const uint32_t lane = threadIdx.x & 63, cm = (1u << rs) - 1u;
    const uint32_t lead = __builtin_amdgcn_readfirstlane(b);
    const unsigned long long same = __ballot(b == lead);
    if (b == lead) {
        if ((int)lane == (int)__ffsll((long long)same) - 1)
            atomicAdd(&h[(lead << rs) + (lane & cm)], (uint32_t)__popcll(same));
    } else {
        atomicAdd(&h[(b << rs) + (lane & cm)], 1u);
    }
}

// ---------------------------------------------------------------- accum --
template <typename TX, typename TY, bool VEC>
__global__ void __launch_bounds__(kT) k_met_accum(const TX *x, const TY *y, int64_t nvox, int nb, int rs,
                                                 const Stats *stp, AccPart *part,
                                                 unsigned long long *hist)
{
    constexpr bool HY = !std::is_same<TY, None>::value;
    extern __shared__ uint32_t lh[];     // [nv][nb][R]; reused for the sums
    const int nv = HY ? 2 : 1, R = 1 << rs;
    for (int i = threadIdx.x; i < nv * nb * R; i += kT) lh[i] = 0u;
    const Stats st = *stp;
    const uint32_t nbm1 = (uint32_t)nb - 1;
    uint32_t *hy = lh + nb * R;
    __syncthreads();
    double sxx = 0.0, syy = 0.0, sdd = 0.0;
    const int64_t nch = nvox / kChunk, stride = (int64_t)gridDim.x * kT;
    // one voxel (pair): deviations from the means and the pair's difference
    auto voxel = [&](float a, float b) {
        const double cx = fma((double)a, st.inv[0], st.off[0]);
        sxx = fma(cx, cx, sxx);
        count_bin(lh, met_bin(a, st.lo[0], st.scale[0], nbm1), rs);
        if constexpr (HY) {
            const double cy = fma((double)b, st.inv[1], st.off[1]);
            syy = fma(cy, cy, syy);
            const double d = (cx - cy) + st.dmean;
            sdd = fma(d, d, sdd);
            count_bin(hy, met_bin(b, st.lo[1], st.scale[1], nbm1), rs);
        }
    };
    for (int64_t c = (int64_t)blockIdx.x * kT + threadIdx.x; c < nch; c += stride) {
        float fx[kChunk], fy[kChunk];
        load8<TX, VEC>(x, c, fx);
        if constexpr (HY) load8<TY, VEC>(y, c, fy);
#pragma unroll
        for (int k = 0; k < kChunk; ++k) voxel(fx[k], HY ? fy[k] : 0.f);
    }
    if (blockIdx.x == gridDim.x - 1) {   // the last work-group takes the tail
        const int64_t t = nch * kChunk + threadIdx.x;
        // whole wavefronts stay together for the ballot in count_bin
        if (t < nvox) {
            float a = (float)x[t], b = 0.f;
            if constexpr (HY) b = (float)y[t];
            voxel(a, b);
        }
    }
    __syncthreads();
    for (int i = threadIdx.x; i < nv * nb; i += kT) {
        uint32_t c = 0;
        for (int r = 0; r < R; ++r) c += lh[i * R + r];
        if (c) atomicAdd(&hist[i], (unsigned long long)c);
    }
    double *red = reinterpret_cast<double *>(lh);   // group_sum waits for the flush
    const double a = group_sum(sxx, red);
    double b = 0.0, d = 0.0;
    if constexpr (HY) {
        b = group_sum(syy, red);
        d = group_sum(sdd, red);
    }
    if (threadIdx.x == 0) part[blockIdx.x] = AccPart{a, b, d, 0.0};
}

// ---------------------------------------------------------------- final --
__global__ void __launch_bounds__(kT) k_met_final(const AccPart *part, int groups, int nv, int64_t nvox,
                                                 int nb, double peak, const Stats *st,
                                                 const unsigned long long *hist,
                                                 mclahe_metrics_result *res, unsigned long long *hist_out)
{
    __shared__ double red[4];
    double sxx = 0.0, syy = 0.0, sdd = 0.0;
    for (int g = threadIdx.x; g < groups; g += kT) {
        sxx += part[g].sxx;
        syy += part[g].syy;
        sdd += part[g].sdd;
    }
    sxx = group_sum(sxx, red);
    syy = group_sum(syy, red);
    sdd = group_sum(sdd, red);
    const double n = (double)nvox;
    double ent[2] = {0.0, 0.0};
    for (int v = 0; v < nv; ++v) {
        double e = 0.0;
        for (int j = threadIdx.x; j < nb; j += kT) {
            const unsigned long long c = hist[v * nb + j];
            if (hist_out) hist_out[v * nb + j] = c;
            if (c) {
                const double p = (double)c / n;
                e -= p * log2(p);
            }
        }
        ent[v] = group_sum(e, red);
    }
    if (threadIdx.x == 0) {
        mclahe_metrics_result r = {};
        for (int v = 0; v < nv; ++v) {
            r.lo[v] = st->lo[v];
            r.hi[v] = st->hi[v];
            r.mean[v] = st->mean[v];
            r.entropy[v] = ent[v];
        }
        r.std[0] = sqrt(sxx / n);
        if (nv == 2) {
            r.std[1] = sqrt(syy / n);
            r.mse = sdd / n;
            r.psnr = r.mse > 0.0 ? 10.0 * log10(peak * peak / r.mse) : INFINITY;
        }
        r.count = (uint64_t)nvox;
        *res = r;
    }
}

// ---------------------------------------------------------------- host --
int met_groups(int64_t nvox)
{
    const int64_t want = (nvox / kChunk + kT * 4 - 1) / (kT * 4);   // >= 4 chunks per thread
    return (int)std::min<int64_t>(kMaxGroups, std::max<int64_t>(1, want));
}

struct MetLayout {
    size_t stats, rpart, apart, hist, total;
};
MetLayout met_layout(int64_t nvox, int nb)
{
    auto a256 = [](size_t v) { return (v + 255) & ~size_t(255); };
    const int g = met_groups(nvox);
    MetLayout L;
    L.stats = 0;
    L.rpart = a256(sizeof(Stats));
    L.apart = L.rpart + a256(sizeof(RangePart) * g);
    L.hist = L.apart + a256(sizeof(AccPart) * g);
    L.total = L.hist + a256(sizeof(unsigned long long) * 2 * nb);
    return L;
}

// parts: NULL, or the nparts min/max/sum records of x and y already written
// by the interpolation units of a CLAHE run (then the range pass is skipped).
template <typename TX, typename TY, bool VEC>
mclahe_status launch_passes(const void *x, const void *y, int64_t nvox, int nb, double peak,
                            mclahe_metrics_result *res, unsigned long long *hist_out, char *ws,
                            hipStream_t st, const RangePart *parts = nullptr, int nparts = 0)
{
    constexpr bool HY = !std::is_same<TY, None>::value;
    const int nv = HY ? 2 : 1, g = met_groups(nvox);
    const MetLayout L = met_layout(nvox, nb);
    Stats *sp = (Stats *)(ws + L.stats);
    RangePart *rp = (RangePart *)(ws + L.rpart);
    AccPart *ap = (AccPart *)(ws + L.apart);
    unsigned long long *h = (unsigned long long *)(ws + L.hist);
    if (parts) {
        hipLaunchKernelGGL(k_met_stats, dim3(1), dim3(kT), 0, st, parts, nparts, nv, nvox, nb, sp, h);
    } else {
        hipLaunchKernelGGL((k_met_range<TX, TY, VEC>), dim3(g), dim3(kT), 0, st, (const TX *)x, (const TY *)y,
                           nvox, rp);
        hipLaunchKernelGGL(k_met_stats, dim3(1), dim3(kT), 0, st, rp, g, nv, nvox, nb, sp, h);
    }
    int rs = 0;   // copies per bin: as many as fit the LDS budget, at most 4
    while ((2 << rs) <= kMaxCopies && sizeof(uint32_t) * nv * nb * (2 << rs) <= kCopyLds) ++rs;
    const size_t lds = std::max(sizeof(uint32_t) * nv * nb * (1 << rs), 4 * sizeof(double));
    hipLaunchKernelGGL((k_met_accum<TX, TY, VEC>), dim3(g), dim3(kT), lds, st,
                       (const TX *)x, (const TY *)y, nvox, nb, rs, sp, ap, h);
    hipLaunchKernelGGL(k_met_final, dim3(1), dim3(kT), 0, st, ap, g, nv, nvox, nb, peak, sp, h, res,
                       hist_out);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "metrics launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

template <typename TX, typename TY>
mclahe_status pick_vec(const void *x, const void *y, int64_t nvox, int nb, double peak,
                       mclahe_metrics_result *res, unsigned long long *hist_out, char *ws, hipStream_t st,
                       const RangePart *parts = nullptr, int nparts = 0)
{
    // vector loads need both bases aligned to one chunk's access width
    auto aligned = [](const void *p, size_t es) {
        const size_t w = es * kChunk >= 16 ? 16 : es * kChunk;
        return ((uintptr_t)p % w) == 0;
    };
    bool vec = aligned(x, sizeof(TX));
    if constexpr (!std::is_same<TY, None>::value) vec = vec && aligned(y, sizeof(TY));
    return vec ? launch_passes<TX, TY, true>(x, y, nvox, nb, peak, res, hist_out, ws, st, parts, nparts)
               : launch_passes<TX, TY, false>(x, y, nvox, nb, peak, res, hist_out, ws, st, parts, nparts);
}

template <typename TX>
mclahe_status pick_y_parts(const void *x, const void *y, int ydt, int64_t nvox, int nb, double peak,
                           mclahe_metrics_result *res, unsigned long long *hist_out, char *ws, hipStream_t st,
                           const RangePart *parts, int nparts)
{
    switch (ydt) {
    case MCLAHE_U8: return pick_vec<TX, uint8_t>(x, y, nvox, nb, peak, res, hist_out, ws, st, parts, nparts);
    case MCLAHE_U16: return pick_vec<TX, uint16_t>(x, y, nvox, nb, peak, res, hist_out, ws, st, parts, nparts);
    default: return pick_vec<TX, float>(x, y, nvox, nb, peak, res, hist_out, ws, st, parts, nparts);
    }
}

template <typename TX>
mclahe_status pick_y(const void *x, const void *y, int ydt, int64_t nvox, int nb, double peak,
                     mclahe_metrics_result *res, unsigned long long *hist_out, char *ws, hipStream_t st)
{
    if (!y) return pick_vec<TX, None>(x, y, nvox, nb, peak, res, hist_out, ws, st);
    switch (ydt) {
    case MCLAHE_U8: return pick_vec<TX, uint8_t>(x, y, nvox, nb, peak, res, hist_out, ws, st);
    case MCLAHE_U16: return pick_vec<TX, uint16_t>(x, y, nvox, nb, peak, res, hist_out, ws, st);
    default: return pick_vec<TX, float>(x, y, nvox, nb, peak, res, hist_out, ws, st);
    }
}

bool valid_dt(int dt) { return dt == MCLAHE_U8 || dt == MCLAHE_U16 || dt == MCLAHE_F32; }

}  // namespace

size_t mc_metrics_tail_ws(int64_t nvox, int n_bins, int nparts)
{
    (void)nparts;   // the records stay where the interpolation units wrote them
    return met_layout(nvox, n_bins).total;
}

mclahe_status mc_metrics_tail(const void *x, int x_dt, const void *y, int y_dt, int64_t nvox, int n_bins,
                              double peak, const McMetPart *parts, int nparts, mclahe_metrics_result *res,
                              uint64_t *hist_out, char *ws, hipStream_t st)
{
    unsigned long long *ho = (unsigned long long *)hist_out;
    switch (x_dt) {
    case MCLAHE_U8: return pick_y_parts<uint8_t>(x, y, y_dt, nvox, n_bins, peak, res, ho, ws, st, parts, nparts);
    case MCLAHE_U16: return pick_y_parts<uint16_t>(x, y, y_dt, nvox, n_bins, peak, res, ho, ws, st, parts, nparts);
    default: return pick_y_parts<float>(x, y, y_dt, nvox, n_bins, peak, res, ho, ws, st, parts, nparts);
    }
}

extern "C" {

mclahe_status mclahe_metrics_workspace_size(int64_t nvox, int n_bins, size_t *bytes)
{
    mc_clear_error();
    if (!bytes) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "bytes is NULL");
    if (nvox < 1) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "nvox must be >= 1 (got %lld)", (long long)nvox);
    if (n_bins < 2 || n_bins > kMaxBins)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "n_bins must be in [2, %d] (got %d)", kMaxBins, n_bins);
    *bytes = met_layout(nvox, n_bins).total;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_metrics(const void *d_x, mclahe_dtype x_dtype, const void *d_y, mclahe_dtype y_dtype,
                             int64_t nvox, int n_bins, double peak, mclahe_metrics_result *d_result,
                             uint64_t *d_hist, void *d_workspace, size_t workspace_bytes, void *hip_stream)
{
    size_t need = 0;
    mclahe_status s = mclahe_metrics_workspace_size(nvox, n_bins, &need);
    if (s) return s;
    if (!d_x || !d_result) return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "x and result must not be NULL");
    if (!valid_dt(x_dtype) || (d_y && !valid_dt(y_dtype)))
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "unknown dtype");
    if (!(peak > 0.0) || !std::isfinite(peak))
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "peak must be positive and finite");
    if (!d_workspace || ((uintptr_t)d_workspace & 255) || workspace_bytes < need)
        return mc_fail(MCLAHE_ERROR_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu at %p)",
                       need, workspace_bytes, d_workspace);
    hipStream_t st = (hipStream_t)hip_stream;
    char *ws = (char *)d_workspace;
    unsigned long long *ho = (unsigned long long *)d_hist;
    switch (x_dtype) {
    case MCLAHE_U8: return pick_y<uint8_t>(d_x, d_y, y_dtype, nvox, n_bins, peak, d_result, ho, ws, st);
    case MCLAHE_U16: return pick_y<uint16_t>(d_x, d_y, y_dtype, nvox, n_bins, peak, d_result, ho, ws, st);
    default: return pick_y<float>(d_x, d_y, y_dtype, nvox, n_bins, peak, d_result, ho, ws, st);
    }
}

}  // extern "C"
