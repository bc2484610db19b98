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
//   - last axis (contiguous), rows of up to 2048 samples: a work-group stages
//     whole rows in LDS, each with its r reflected halo samples on both
//     sides, and every output reads its taps at fixed offsets;
//   - longer rows: a flat tile of 2048 outputs plus r halo samples on each
//     side (reflection never reaches further than r from an output);
//   - the last two axes, both smoothed, rows of at most 512 samples: one
//     fused pass through LDS (k_gauss_last2);
//   - two consecutive smoothed axes before those, both strided, radii up to
//     8: one pass (k_gauss_pair), the first axis in a register ring per
//     thread, the second through LDS;
//   - any other axis (stride S): a thread owns 4 (or 1) adjacent columns and
//     sweeps a segment of the axis with a ring of 2r + 1 samples in
//     registers, unrolled by the ring length so that every slot index is a
//     compile-time constant: each input is loaded once per segment.
// Median: values become order-preserving unsigned keys (integer min/max);
// a bitonic network padded to a power of two sorts them and the key of rank
// N / 2 (0-based) is written back in the input dtype.  Two launches: outputs
// whose window lies inside the array (4 consecutive outputs of a row per
// thread where the window allows, values gathered at precomputed flat
// offsets), then the border slabs (coordinates reflected per value).
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
// Taps of output position p (of a row of n) whose window crosses a row end:
// one reflection suffices while r < n, repeated reflection otherwise.
__device__ __forceinline__ int tap_pos(int q, int n, bool single)
{
    if (single) {
        q = q < 0 ? -q - 1 : q;
        return q >= n ? 2 * n - 1 - q : q;
    }
    return (int)refl(q, n);
}

// RT > 0: the radius as a compile-time constant (taps unrolled, weights in
// registers); RT = 0: any radius r.
template <typename T, int RT>
__global__ void __launch_bounds__(kT) k_gauss_last(const T *in, float *out, int64_t nvox, int64_t n, int r,
                                                  Weights W)
{
    if constexpr (RT > 0) r = RT;
    extern __shared__ float tile[];   // [kTile + 2r]
    const int64_t e0 = (int64_t)blockIdx.x * kTile;
    const int64_t lo = e0 - r;
    const int len = kTile + 2 * r;
    {
        float v[kTile / kT];          // all of a thread's loads in flight at once
#pragma unroll
        for (int k = 0; k < kTile / kT; ++k) {
            const int64_t e = lo + threadIdx.x + k * kT;
            v[k] = (e >= 0 && e < nvox) ? ld1(in, e) : 0.f;
        }
#pragma unroll
        for (int k = 0; k < kTile / kT; ++k) tile[threadIdx.x + k * kT] = v[k];
        for (int i = kTile + threadIdx.x; i < len; i += kT) {
            const int64_t e = lo + i;
            tile[i] = (e >= 0 && e < nvox) ? ld1(in, e) : 0.f;
        }
    }
    float w[RT > 0 ? 2 * RT + 1 : 1];
    if constexpr (RT > 0) {
#pragma unroll
        for (int j = 0; j <= 2 * RT; ++j) w[j] = W.w[j];
    }
    __syncthreads();
    // position in its row of the thread's first output, then stepped by kT
    // (all 32-bit: rows of up to 2^30 samples)
    const int nn = (int)n;
    const int step = kT % nn;
    int p = (int)((e0 + threadIdx.x) % n);
    const bool single = r < nn;
#pragma unroll 2
    for (int k = 0; k < kTile / kT; ++k) {
        const int t = threadIdx.x + k * kT;
        const int64_t e = e0 + t;
        if (e >= nvox) break;
        float acc = 0.f;
        if (p >= r && p + r < nn) {
            if constexpr (RT > 0) {
#pragma unroll
                for (int j = 0; j <= 2 * RT; ++j) acc = __builtin_fmaf(w[j], tile[t + j], acc);
            } else {
                for (int j = 0; j <= 2 * r; ++j) acc = __builtin_fmaf(W.w[j], tile[t + j], acc);
            }
        } else {
            // same row, within r of e: tile index t + r + (q - p)
            for (int j = -r; j <= r; ++j) {
                const int q = tap_pos(p + j, nn, single);
                acc = __builtin_fmaf(W.w[j + r], tile[t + r + q - p], acc);
            }
        }
        out[e] = acc;
        p += step;
        if (p >= nn) p -= nn;
    }
}

// Short rows (n <= kTile): a work-group stages whole rows, each with its r
// reflected halo samples on both sides, so that every output reads its taps
// at fixed offsets (no per-output reflection, no divergence at row ends).
template <typename T, int RT>
__global__ void __launch_bounds__(kT) k_gauss_rows(const T *in, float *out, int64_t nvox, int n, int r,
                                                  int rows_per_group, Weights W)
{
    if constexpr (RT > 0) r = RT;
    extern __shared__ float rowbuf[];   // [rows][n + 2r]
    const int rs = n + 2 * r;
    const int64_t e0 = (int64_t)blockIdx.x * rows_per_group * n;
    const int cnt = (int)std::min<int64_t>((int64_t)rows_per_group * n, nvox - e0);
    const int dr = kT / n, dp = kT % n;
    {
        // 8 loads per thread in flight before they are stored
        int row = threadIdx.x / n, p = threadIdx.x % n;
        for (int i0 = threadIdx.x; i0 < cnt; i0 += 8 * kT) {
            float v[8];
            int slot[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                if (i0 + k * kT < cnt) v[k] = ld1(in, e0 + i0 + k * kT);
                slot[k] = row * rs + r + p;
                row += dr;
                p += dp;
                if (p >= n) {
                    p -= n;
                    ++row;
                }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (i0 + k * kT < cnt) rowbuf[slot[k]] = v[k];
        }
    }
    __syncthreads();
    const int rows = cnt / n;
    for (int h = threadIdx.x; h < rows * 2 * r; h += kT) {
        const int row = h / (2 * r), sl = h - row * 2 * r;
        const int q = sl < r ? sl - r : n + (sl - r);          // position of the halo slot
        rowbuf[row * rs + r + q] = rowbuf[row * rs + r + tap_pos(q, n, r < n)];
    }
    __syncthreads();
    float w[RT > 0 ? 2 * RT + 1 : 1];
    if constexpr (RT > 0) {
#pragma unroll
        for (int j = 0; j <= 2 * RT; ++j) w[j] = W.w[j];
    }
    int row = threadIdx.x / n, p = threadIdx.x % n;
    for (int i = threadIdx.x; i < cnt; i += kT) {
        const float *src = rowbuf + row * rs + p;   // taps p - r .. p + r
        float acc = 0.f;
        if constexpr (RT > 0) {
#pragma unroll
            for (int j = 0; j <= 2 * RT; ++j) acc = __builtin_fmaf(w[j], src[j], acc);
        } else {
            for (int j = 0; j <= 2 * r; ++j) acc = __builtin_fmaf(W.w[j], src[j], acc);
        }
        out[e0 + i] = acc;
        row += dr;
        p += dp;
        if (p >= n) {
            p -= n;
            ++row;
        }
    }
}

// Minimum and maximum over the work-group (kT threads) to dst[0], dst[1].
__device__ __forceinline__ void block_minmax(float mn, float mx, float *dst)
{
    __shared__ float red[2][kT / 64];
    for (int o = 32; o > 0; o >>= 1) {
        mn = fminf(mn, __shfl_xor(mn, o));
        mx = fmaxf(mx, __shfl_xor(mx, o));
    }
    if ((threadIdx.x & 63) == 0) {
        red[0][threadIdx.x >> 6] = mn;
        red[1][threadIdx.x >> 6] = mx;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < kT / 64; ++w) {
            red[0][0] = fminf(red[0][0], red[0][w]);
            red[1][0] = fmaxf(red[1][0], red[1][w]);
        }
        dst[0] = red[0][0];
        dst[1] = red[1][0];
    }
}

// (min, max) pairs [b n / m, (b + 1) n / m) of src -> pair b of dst, for
// b < m work-groups.
__global__ void __launch_bounds__(kT) k_minmax_reduce(const float *src, int64_t n, float *dst, uint32_t m)
{
    const int64_t a = n * blockIdx.x / m, b = n * (blockIdx.x + 1) / m;
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t i = a + threadIdx.x; i < b; i += kT) {
        mn = fminf(mn, src[2 * i]);
        mx = fmaxf(mx, src[2 * i + 1]);
    }
    block_minmax(mn, mx, dst + 2 * (int64_t)blockIdx.x);
}

// The last two axes in one pass (both smoothed, rows of at most kFuseRow
// samples): a work-group takes T2 consecutive rows along axis D-2 of one
// outer index, loads them with r2 halo rows on each side (reflected along
// axis D-2) into LDS, filters along axis D-2 into a second LDS buffer laid
// out with r3 halo slots per row, fills those by reflection along the last
// axis and filters along it.  The same chains as two separate passes, so
// the result is identical; one round trip through HBM less.
constexpr int kFuseRow = 512;
constexpr int kFuseRowTab = kTile / 2 + 2 * kRadiusMax;       // rows a group loads, at most
// dynamic LDS of a group: 64 KiB less the row table and the min/max scratch
constexpr size_t kFuseLds = 65536 - sizeof(int) * kFuseRowTab - sizeof(float) * 2 * (kT / 64);

// mm: NULL, or room for one (min, max) pair of the outputs per work-group
// (the global range of the smoothed volume, reduced later).
template <typename T, int R2, int R3>
__global__ void __launch_bounds__(kT) k_gauss_last2(const T *in, float *out, int n2, int n3, int r2, int r3,
                                                   int T2, Weights W2, Weights W3, float *mm)
{
    if constexpr (R2 > 0) r2 = R2;
    if constexpr (R3 > 0) r3 = R3;
    extern __shared__ float4 lds4[];                      // 16-byte aligned
    float *lds = reinterpret_cast<float *>(lds4);
    __shared__ int rowsrc[kFuseRowTab];   // offset of the source row of each loaded row
    const int nseg = (n2 + T2 - 1) / T2;
    const int64_t outer = blockIdx.x / nseg;
    const int q0 = (int)(blockIdx.x - outer * nseg) * T2;
    const int rows = min(T2, n2 - q0);            // output rows of this group
    const int la = rows + 2 * r2;                 // loaded rows
    const int rs = n3 + 2 * r3;
    float *A = lds;                               // [la][n3]
    float *B = lds + (size_t)(T2 + 2 * r2) * n3;  // [rows][n3 + 2 r3]
    const T *src = in + outer * (int64_t)n2 * n3;
    for (int t = threadIdx.x; t < la; t += kT) rowsrc[t] = tap_pos(q0 - r2 + t, n2, r2 < n2) * n3;
    __syncthreads();
    // (row, position) of element i = threadIdx.x + k kT, stepped without
    // divisions
    const int t00 = threadIdx.x / n3, p00 = threadIdx.x - t00 * n3;
    const int dt = kT / n3, dp = kT - dt * n3;
    const int total = la * n3;
    if (sizeof(T) == 4 && (n3 & 3) == 0 && ((uintptr_t)src & 15) == 0) {
        // 16-byte loads: element quads (row t, positions 4c .. 4c+3)
        const int nq = n3 >> 2, tq = threadIdx.x / nq, cq = threadIdx.x - tq * nq;
        const int dtq = kT / nq, dcq = kT - dtq * nq;
        int t = tq, c = cq;
        for (int j0 = threadIdx.x; j0 < total / 4; j0 += 4 * kT) {
            float4 v[4];
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                v[k] = make_float4(0.f, 0.f, 0.f, 0.f);
                if (j0 + k * kT < total / 4)
                    v[k] = *reinterpret_cast<const float4 *>(reinterpret_cast<const float *>(src) + rowsrc[t] + 4 * c);
                t += dtq;
                c += dcq;
                if (c >= nq) { c -= nq; ++t; }
            }
#pragma unroll
            for (int k = 0; k < 4; ++k)
                if (j0 + k * kT < total / 4) reinterpret_cast<float4 *>(A)[j0 + k * kT] = v[k];
        }
    } else {
        int t = t00, p = p00;
        for (int i0 = threadIdx.x; i0 < total; i0 += 8 * kT) {
            float v[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) {
                v[k] = 0.f;
                if (i0 + k * kT < total) v[k] = ld1(src, rowsrc[t] + p);
                t += dt;
                p += dp;
                if (p >= n3) { p -= n3; ++t; }
            }
#pragma unroll
            for (int k = 0; k < 8; ++k)
                if (i0 + k * kT < total) A[i0 + k * kT] = v[k];
        }
    }
    __syncthreads();
    float w2[R2 > 0 ? 2 * R2 + 1 : 1];
    if constexpr (R2 > 0) {
#pragma unroll
        for (int j = 0; j <= 2 * R2; ++j) w2[j] = W2.w[j];
    }
    int t = t00, p = p00;
    for (int i = threadIdx.x; i < rows * n3; i += kT) {
        float acc = 0.f;
        if constexpr (R2 > 0) {
#pragma unroll
            for (int j = 0; j <= 2 * R2; ++j) acc = __builtin_fmaf(w2[j], A[(t + j) * n3 + p], acc);
        } else {
            for (int j = 0; j <= 2 * r2; ++j) acc = __builtin_fmaf(W2.w[j], A[(t + j) * n3 + p], acc);
        }
        B[t * rs + r3 + p] = acc;
        t += dt;
        p += dp;
        if (p >= n3) { p -= n3; ++t; }
    }
    __syncthreads();
    for (int h = threadIdx.x; h < rows * 2 * r3; h += kT) {
        const int t = h / (2 * r3), sl = h - t * 2 * r3;
        const int q = sl < r3 ? sl - r3 : n3 + (sl - r3);
        B[t * rs + r3 + q] = B[t * rs + r3 + tap_pos(q, n3, r3 < n3)];
    }
    __syncthreads();
    float w3[R3 > 0 ? 2 * R3 + 1 : 1];
    if constexpr (R3 > 0) {
#pragma unroll
        for (int j = 0; j <= 2 * R3; ++j) w3[j] = W3.w[j];
    }
    const int64_t ob = outer * (int64_t)n2 * n3 + (int64_t)q0 * n3;
    t = t00;
    p = p00;
    float mn = INFINITY, mx = -INFINITY;
    for (int i = threadIdx.x; i < rows * n3; i += kT) {
        const float *src = B + t * rs + p;
        float acc = 0.f;
        if constexpr (R3 > 0) {
#pragma unroll
            for (int j = 0; j <= 2 * R3; ++j) acc = __builtin_fmaf(w3[j], src[j], acc);
        } else {
            for (int j = 0; j <= 2 * r3; ++j) acc = __builtin_fmaf(W3.w[j], src[j], acc);
        }
        out[ob + i] = acc;
        mn = fminf(mn, acc);
        mx = fmaxf(mx, acc);
        t += dt;
        p += dp;
        if (p >= n3) { p -= n3; ++t; }
    }
    if (mm) block_minmax(mn, mx, mm + 2 * (int64_t)blockIdx.x);
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
        // the chunk's WN new inputs are loaded back to back (all in flight),
        // then moved into the ring as the outputs consume them
        VecF<V> nxt[WN];
#pragma unroll
        for (int u = 0; u < WN; ++u)
            if (pb + u < p1) nxt[u] = ldv<T, V>(in, base + refl(pb + u + R, c.n) * c.S);
#pragma unroll
        for (int u = 0; u < WN; ++u) {
            const int64_t p = pb + u;
            if (p < p1) {
                ring[(u + 2 * R) % WN] = nxt[u];
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

// Two consecutive strided axes in one pass.  The array is [outer][n0][n1][S]
// (S > 1 elements after the second axis).  A work-group owns a tile of the
// second axis, TY outputs plus r1 halo rows on each side (kPairRows rows in
// all), times kPairCols columns of V adjacent inner elements, and sweeps a
// segment of the first axis.  Every thread smooths its (row, column) along
// the first axis with a ring of 2 R0 + 1 inputs in registers, exactly the
// chain of the one-axis pass; the rows of that plane meet in LDS, and the TY
// output rows are smoothed along the second axis from there, again with the
// one-axis chain (tap positions reflected as that pass reflects them).  The
// result is bit-identical to the two one-axis passes, with one trip through
// HBM instead of two (the halo rows are read twice, mostly from L2).
struct Pair {
    int64_t n0, n1, S;        // first and second axis, inner elements
    int64_t ccols, nty;       // column groups per row, row tiles
    int64_t seg, nseg;        // first-axis positions per segment, segments
    int TY, r1;               // output rows per tile, radius on the second axis
};
constexpr int kPairRows = 32, kPairCols = kT / kPairRows;

template <typename T, int V, int R0>
__global__ void __launch_bounds__(kT) k_gauss_pair(const T *in, float *out, Pair g, Weights W0, Weights W1)
{
    constexpr int WN = 2 * R0 + 1;
    constexpr int CW = kPairCols * V;            // floats per LDS row
    __shared__ __align__(16) float tl[kPairRows][CW];
    int64_t b = blockIdx.x;
    const int64_t cc = b % g.ccols;
    b /= g.ccols;
    const int64_t ty = b % g.nty;
    b /= g.nty;
    const int64_t sg = b % g.nseg;
    const int64_t ou = b / g.nseg;
    const int row = threadIdx.x / kPairCols, cx = threadIdx.x % kPairCols;
    const int64_t s = (cc * kPairCols + cx) * V;
    const bool colok = s < g.S;                  // V divides S
    const int64_t y = ty * g.TY + row - g.r1;    // second-axis position of the row
    const int64_t pst = g.n1 * g.S;              // first-axis stride
    const int64_t ibase = ou * g.n0 * pst + refl(y, g.n1) * g.S + s;
    const bool outrow = colok && row >= g.r1 && row < g.r1 + g.TY && y < g.n1;
    const int64_t obase = ou * g.n0 * pst + y * g.S + s;
    const int64_t p0 = sg * g.seg, p1 = std::min(p0 + g.seg, g.n0);
    float w[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j) w[j] = W0.w[j];
    VecF<V> ring[WN];
#pragma unroll
    for (int j = 0; j < WN; ++j)
#pragma unroll
        for (int k = 0; k < V; ++k) ring[j].v[k] = 0.f;
    // slot of first-axis position q: (q - (p0 - R0)) mod WN
#pragma unroll
    for (int j = 0; j < 2 * R0; ++j)
        if (colok) ring[j] = ldv<T, V>(in, ibase + refl(p0 - R0 + j, g.n0) * pst);
    for (int64_t pb = p0; pb < p1; pb += WN) {
        VecF<V> nxt[WN];
#pragma unroll
        for (int u = 0; u < WN; ++u) {
#pragma unroll
            for (int k = 0; k < V; ++k) nxt[u].v[k] = 0.f;
            if (colok && pb + u < p1) nxt[u] = ldv<T, V>(in, ibase + refl(pb + u + R0, g.n0) * pst);
        }
#pragma unroll
        for (int u = 0; u < WN; ++u) {
            const int64_t p = pb + u;
            if (p < p1) {                        // the same for the whole work-group
                ring[(u + 2 * R0) % WN] = nxt[u];
                float acc[V];
#pragma unroll
                for (int k = 0; k < V; ++k) acc[k] = 0.f;
#pragma unroll
                for (int j = 0; j < WN; ++j)
#pragma unroll
                    for (int k = 0; k < V; ++k) acc[k] = __builtin_fmaf(w[j], ring[(u + j) % WN].v[k], acc[k]);
#pragma unroll
                for (int k = 0; k < V; ++k) tl[row][cx * V + k] = acc[k];
                __syncthreads();
                if (outrow) {
                    float o[V];
#pragma unroll
                    for (int k = 0; k < V; ++k) o[k] = 0.f;
                    for (int j = 0; j <= 2 * g.r1; ++j)
#pragma unroll
                        for (int k = 0; k < V; ++k) o[k] = __builtin_fmaf(W1.w[j], tl[row - g.r1 + j][cx * V + k], o[k]);
                    stv<V>(out, obase + p * pst, o);
                }
                __syncthreads();
            }
        }
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
    int64_t off[kMedianMax];         // flat offset of window value i (interior outputs)
    int8_t woff[kMedianMax][MC_MAXD];  // per-axis offset of window value i
    // border slabs: along axis a, positions [0, b0[a]) and [shape - b1[a], shape)
    // (all positions if they meet), times every position of the other axes
    int64_t b0[MC_MAXD], b1[MC_MAXD], slab_pre[MC_MAXD + 1];
};

// Order-preserving unsigned keys (integer min/max, no float canonicalising).
template <typename T> __device__ __forceinline__ uint32_t key_of(T v) { return (uint32_t)v; }
template <> __device__ __forceinline__ uint32_t key_of<float>(float v)
{
    const uint32_t u = __float_as_uint(v);
    return (u & 0x80000000u) ? ~u : (u | 0x80000000u);
}
template <typename T> __device__ __forceinline__ T val_of(uint32_t k) { return (T)k; }
template <> __device__ __forceinline__ float val_of<float>(uint32_t k)
{
    return __uint_as_float((k & 0x80000000u) ? (k & 0x7fffffffu) : ~k);
}

template <typename T, int V>
__device__ __forceinline__ void ldk(const T *p, int64_t i, uint32_t (&k)[V])
{
    if constexpr (V == 4 && sizeof(T) == 4) {
        const float4 a = *reinterpret_cast<const float4 *>(p + i);
        k[0] = key_of<float>(a.x); k[1] = key_of<float>(a.y); k[2] = key_of<float>(a.z); k[3] = key_of<float>(a.w);
    } else if constexpr (V == 4 && sizeof(T) == 2) {
        const uint2 a = *reinterpret_cast<const uint2 *>(p + i);
        k[0] = a.x & 0xffffu; k[1] = a.x >> 16; k[2] = a.y & 0xffffu; k[3] = a.y >> 16;
    } else if constexpr (V == 4 && sizeof(T) == 1) {
        const uint32_t a = *reinterpret_cast<const uint32_t *>(p + i);
#pragma unroll
        for (int j = 0; j < 4; ++j) k[j] = (a >> (8 * j)) & 0xffu;
    } else {
#pragma unroll
        for (int j = 0; j < V; ++j) k[j] = key_of<T>(p[i + j]);
    }
}

template <int NP>
__device__ __forceinline__ void bitonic_sort(uint32_t (&a)[NP])
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
                    const uint32_t x = a[i], y = a[j];
                    a[i] = up ? min(x, y) : max(x, y);
                    a[j] = up ? max(x, y) : min(x, y);
                }
            }
}

// Key of rank `rank` among NP keys (padding keys are all ones: they sort last).
template <int NP, bool EXACT>
__device__ __forceinline__ uint32_t rank_key(uint32_t (&v)[NP], int rank)
{
    bitonic_sort<NP>(v);
    if constexpr (EXACT) return v[NP / 2];
    uint32_t m = v[0];
#pragma unroll
    for (int i = 0; i < NP; ++i)
        if (i == rank) m = v[i];
    return m;
}

template <typename T, int VM>
__device__ __forceinline__ void stk(T *p, int64_t i, const uint32_t (&m)[VM])
{
    if constexpr (VM == 4 && sizeof(T) == 4) {
        *reinterpret_cast<float4 *>(p + i) =
            make_float4(val_of<float>(m[0]), val_of<float>(m[1]), val_of<float>(m[2]), val_of<float>(m[3]));
    } else if constexpr (VM == 4 && sizeof(T) == 2) {
        *reinterpret_cast<uint2 *>(p + i) = make_uint2(m[0] | (m[1] << 16), m[2] | (m[3] << 16));
    } else if constexpr (VM == 4 && sizeof(T) == 1) {
        *reinterpret_cast<uint32_t *>(p + i) = m[0] | (m[1] << 8) | (m[2] << 16) | (m[3] << 24);
    } else {
#pragma unroll
        for (int j = 0; j < VM; ++j) p[i + j] = val_of<T>(m[j]);
    }
}

// Outputs whose window lies inside the array: VM consecutive outputs of one
// row per thread (VM = 4 needs a last-axis window of 1, a row length
// divisible by 4 and aligned bases), window values gathered at precomputed
// flat offsets.  Outputs near a border are left to k_median_border.  EXACT:
// the window holds NP values.  IX: type of the coordinate arithmetic
// (32-bit for arrays under 2^31 voxels).
template <typename T, int NP, int VM, bool EXACT, typename IX>
__global__ void __launch_bounds__(kT) k_median_interior(const T *in, T *out, MedGeom g)
{
    const int64_t e0 = ((int64_t)blockIdx.x * kT + threadIdx.x) * VM;
    if (e0 >= g.nvox) return;
    IX rem = (IX)e0;
    bool interior = true;
#pragma unroll
    for (int a = 0; a < MC_MAXD; ++a)
        if (a < g.D) {
            const IX st = (IX)g.stride[a];
            const IX pa = rem / st;
            rem -= pa * st;
            const int64_t q0 = (int64_t)pa + g.lo[a];
            const int64_t q1 = q0 + g.k[a] - 1 + (a == g.D - 1 ? VM - 1 : 0);
            interior = interior && (g.k[a] == 1 || (q0 >= 0 && q1 < g.shape[a]));
        }
    if (!interior) return;
    uint32_t x[NP][VM];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        if (EXACT || i < g.N) ldk<T, VM>(in, e0 + g.off[i], x[i]);
        else {
#pragma unroll
            for (int j = 0; j < VM; ++j) x[i][j] = 0xffffffffu;
        }
    }
    uint32_t m[VM];
#pragma unroll
    for (int j = 0; j < VM; ++j) {
        uint32_t v[NP];
#pragma unroll
        for (int i = 0; i < NP; ++i) v[i] = x[i][j];
        m[j] = rank_key<NP, EXACT>(v, g.N / 2);
    }
    stk<T, VM>(out, e0, m);
}

// Outputs near a border: one per thread over the border slabs (a voxel on
// several slabs is computed by each, with the same value), coordinates
// reflected per window value.
template <typename T, int NP>
__global__ void __launch_bounds__(kT) k_median_border(const T *in, T *out, MedGeom g)
{
    const int64_t t = (int64_t)blockIdx.x * kT + threadIdx.x;
    if (t >= g.slab_pre[g.D]) return;
    int s = 0;
#pragma unroll
    for (int a = 1; a < MC_MAXD; ++a)
        if (a < g.D && t >= g.slab_pre[a]) s = a;
    // position along the slab axis, then the other axes from the rest
    const int64_t per = g.nvox / g.shape[s];
    int64_t l = t - g.slab_pre[s];
    const int64_t bi = l / per;
    l -= bi * per;
    const int64_t cnt = g.b0[s] + g.b1[s];
    const int64_t ps = cnt >= g.shape[s] ? bi : (bi < g.b0[s] ? bi : g.shape[s] - cnt + bi);
    int64_t pos[MC_MAXD];
    int64_t rest = l, e = 0;
#pragma unroll
    for (int a = MC_MAXD - 1; a >= 0; --a)
        if (a < g.D) {
            if (a == s) {
                pos[a] = ps;
            } else {
                pos[a] = rest % g.shape[a];
                rest /= g.shape[a];
            }
            e += pos[a] * g.stride[a];
        } else {
            pos[a] = 0;
        }
    uint32_t v[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) {
        v[i] = 0xffffffffu;
        if (i < g.N) {
            int64_t off = 0;
#pragma unroll
            for (int a = 0; a < MC_MAXD; ++a)
                if (a < g.D) off += refl(pos[a] + g.woff[i][a], g.shape[a]) * g.stride[a];
            v[i] = key_of<T>(in[off]);
        }
    }
    out[e] = val_of<T>(rank_key<NP, false>(v, g.N / 2));
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
    if (S == 1 && n <= kTile) {
        // rows per work-group: about kTile outputs, at most 64 KiB of LDS
        const int rpg = (int)std::max<int64_t>(1, std::min<int64_t>(kTile / n, 16384 / (n + 2 * r)));
        const int64_t rows = nvox / n;
        const int64_t blocks = (rows + rpg - 1) / rpg;
        if (blocks > 0x7fffffff) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large for one pass");
        const dim3 grid((uint32_t)blocks), blk(kT);
        const size_t lds = sizeof(float) * rpg * (n + 2 * r);
#define ROWS(RR) \
    case RR: hipLaunchKernelGGL((k_gauss_rows<T, RR>), grid, blk, lds, st, in, out, nvox, (int)n, r, rpg, W); break;
        switch (r) {
            ROWS(1) ROWS(2) ROWS(3) ROWS(4) ROWS(5) ROWS(6) ROWS(7) ROWS(8)
        default: hipLaunchKernelGGL((k_gauss_rows<T, 0>), grid, blk, lds, st, in, out, nvox, (int)n, r, rpg, W);
        }
#undef ROWS
    } else if (S == 1) {
        const int64_t blocks = (nvox + kTile - 1) / kTile;
        if (n > (1 << 30)) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "last axis longer than 2^30");
        const dim3 grid((uint32_t)blocks), blk(kT);
        const size_t lds = sizeof(float) * (kTile + 2 * r);
#define LAST(RR) \
    case RR: hipLaunchKernelGGL((k_gauss_last<T, RR>), grid, blk, lds, st, in, out, nvox, n, r, W); break;
        switch (r) {
            LAST(1) LAST(2) LAST(3) LAST(4) LAST(5) LAST(6) LAST(7) LAST(8)
        default: hipLaunchKernelGGL((k_gauss_last<T, 0>), grid, blk, lds, st, in, out, nvox, n, r, W);
        }
#undef LAST
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
        static_assert(kRingMax == 8, "the ring launches below cover radii 1..8");
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

// Whether two consecutive strided axes (radii r0, r1) go in one pass.
bool pair_ok(int r0, int r1) { return r0 >= 1 && r0 <= kRingMax && r1 >= 1 && r1 <= kRingMax; }

template <typename T>
mclahe_status gauss_pair(const T *in, float *out, int64_t nvox, int64_t n0, int64_t n1, int64_t S, int r0,
                         const Weights &W0, int r1, const Weights &W1, hipStream_t st)
{
    const bool vec = S % 4 == 0 && ((uintptr_t)in % (4 * sizeof(T))) == 0 && ((uintptr_t)out % 16) == 0;
    const int V = vec ? 4 : 1;
    Pair g;
    g.n0 = n0;
    g.n1 = n1;
    g.S = S;
    g.r1 = r1;
    g.TY = kPairRows - 2 * r1;
    g.nty = (n1 + g.TY - 1) / g.TY;
    g.ccols = (S + kPairCols * V - 1) / (kPairCols * V);
    const int64_t outer = nvox / (n0 * n1 * S);
    // segments of the first axis: a multiple of the ring length near 64
    // positions, fewer if the tiles alone do not fill the chip
    const int WN = 2 * r0 + 1;
    int64_t seg = ((64 + WN - 1) / WN) * WN;
    const int64_t tiles = outer * g.nty * g.ccols;
    while (seg > WN && tiles * ((n0 + seg - 1) / seg) < 4096) seg -= WN;
    g.seg = std::min<int64_t>(seg, n0);
    g.nseg = (n0 + g.seg - 1) / g.seg;
    const int64_t blocks = tiles * g.nseg;
    if (blocks > 0x7fffffff) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large for one pass");
    const dim3 grid((uint32_t)blocks), blk(kT);
#define PAIR(RR)                                                                                  \
    case RR:                                                                                      \
        if (vec) hipLaunchKernelGGL((k_gauss_pair<T, 4, RR>), grid, blk, 0, st, in, out, g, W0, W1); \
        else hipLaunchKernelGGL((k_gauss_pair<T, 1, RR>), grid, blk, 0, st, in, out, g, W0, W1);     \
        break;
    switch (r0) {
        PAIR(1) PAIR(2) PAIR(3) PAIR(4) PAIR(5) PAIR(6) PAIR(7) PAIR(8)
    default: return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "pair pass radius");
    }
#undef PAIR
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "gaussian pass launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

// Rows of T2 per work-group for the fused last-two-axes pass: about kTile
// outputs, LDS within 64 KiB.
int fuse_rows(int n2, int n3, int r2, int r3)
{
    // at most kTile / 2 rows: the row table of the kernel holds T2 + 2 r2
    int T2 = std::max(1, std::min({n2, kTile / n3, kTile / 2}));
    while (T2 > 1 && sizeof(float) * ((size_t)(T2 + 2 * r2) * n3 + (size_t)T2 * (n3 + 2 * r3)) > kFuseLds) --T2;
    return T2;
}

template <typename T>
mclahe_status gauss_last2(const T *in, float *out, int64_t nvox, int n2, int n3, int r2, int r3, const Weights &W2,
                          const Weights &W3, hipStream_t st, float *mm)
{
    const int T2 = fuse_rows(n2, n3, r2, r3);
    const int64_t outer = nvox / ((int64_t)n2 * n3);
    const int64_t blocks = outer * ((n2 + T2 - 1) / T2);
    if (blocks > 0x7fffffff) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large for one pass");
    const size_t lds = sizeof(float) * ((size_t)(T2 + 2 * r2) * n3 + (size_t)T2 * (n3 + 2 * r3));
    const dim3 grid((uint32_t)blocks), blk(kT);
    // common radii as constants; any other pair runs the generic loops
    if (r2 == 3 && r3 == 3) hipLaunchKernelGGL((k_gauss_last2<T, 3, 3>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    else if (r2 == 4 && r3 == 5) hipLaunchKernelGGL((k_gauss_last2<T, 4, 5>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    else if (r2 == 3 && r3 == 4) hipLaunchKernelGGL((k_gauss_last2<T, 3, 4>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    else if (r2 == 4 && r3 == 4) hipLaunchKernelGGL((k_gauss_last2<T, 4, 4>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    else if (r2 == 5 && r3 == 5) hipLaunchKernelGGL((k_gauss_last2<T, 5, 5>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    else hipLaunchKernelGGL((k_gauss_last2<T, 0, 0>), grid, blk, lds, st, in, out, n2, n3, r2, r3, T2, W2, W3, mm);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "gaussian pass launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

template <typename T, int NP, typename IX>
void median_launch_np(const void *in, void *out, const MedGeom &g, bool vec, hipStream_t st)
{
    const T *i = (const T *)in;
    T *o = (T *)out;
    const bool exact = g.N == NP;
    if constexpr (NP <= 8) {
        if (vec) {
            const dim3 grid((uint32_t)((g.nvox / 4 + kT - 1) / kT));
            if (exact) hipLaunchKernelGGL((k_median_interior<T, NP, 4, true, IX>), grid, dim3(kT), 0, st, i, o, g);
            else hipLaunchKernelGGL((k_median_interior<T, NP, 4, false, IX>), grid, dim3(kT), 0, st, i, o, g);
            goto border;
        }
    }
    {
        const dim3 grid((uint32_t)((g.nvox + kT - 1) / kT));
        if (exact) hipLaunchKernelGGL((k_median_interior<T, NP, 1, true, IX>), grid, dim3(kT), 0, st, i, o, g);
        else hipLaunchKernelGGL((k_median_interior<T, NP, 1, false, IX>), grid, dim3(kT), 0, st, i, o, g);
    }
border:
    if (g.slab_pre[g.D] > 0)
        hipLaunchKernelGGL((k_median_border<T, NP>), dim3((uint32_t)((g.slab_pre[g.D] + kT - 1) / kT)), dim3(kT), 0,
                           st, i, o, g);
}

template <typename T>
mclahe_status median_launch(const void *in, void *out, const MedGeom &g, hipStream_t st)
{
    const int last = g.D - 1;
    const bool vec = g.N <= 8 && g.k[last] == 1 && g.shape[last] % 4 == 0 &&
                     ((uintptr_t)in % (4 * sizeof(T))) == 0 && ((uintptr_t)out % (4 * sizeof(T))) == 0;
    if (g.nvox >= (1LL << 31)) {
        if (g.N <= 8) median_launch_np<T, 8, uint64_t>(in, out, g, vec, st);
        else median_launch_np<T, 64, uint64_t>(in, out, g, false, st);
    } else if (g.N <= 2) median_launch_np<T, 2, uint32_t>(in, out, g, vec, st);
    else if (g.N <= 4) median_launch_np<T, 4, uint32_t>(in, out, g, vec, st);
    else if (g.N <= 8) median_launch_np<T, 8, uint32_t>(in, out, g, vec, st);
    else if (g.N <= 16) median_launch_np<T, 16, uint32_t>(in, out, g, false, st);
    else if (g.N <= 32) median_launch_np<T, 32, uint32_t>(in, out, g, false, st);
    else median_launch_np<T, 64, uint32_t>(in, out, g, false, st);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return mc_fail(MCLAHE_ERROR_HIP, "median launch failed: %s", hipGetErrorString(e));
    return MCLAHE_SUCCESS;
}

}  // namespace

// Axes a Gaussian call smooths, and whether its last two go in one fused
// pass (both smoothed, short rows, one row group within the LDS budget).
static void gauss_axes(int ndim, const int64_t *shape, const double *sigma, double truncate, std::vector<int> &axes,
                       bool &fuse)
{
    axes.clear();
    for (int i = 0; i < ndim; ++i)
        if (sigma[i] > 0.0) axes.push_back(i);
    const int P = (int)axes.size();
    fuse = P >= 2 && axes[P - 1] == ndim - 1 && axes[P - 2] == ndim - 2 && shape[ndim - 1] <= kFuseRow;
    if (fuse) {
        const int64_t n3 = shape[ndim - 1];
        const int r2 = gauss_radius(sigma[ndim - 2], truncate), r3 = gauss_radius(sigma[ndim - 1], truncate);
        fuse = sizeof(float) * ((1 + 2 * r2) * n3 + (n3 + 2 * r3)) <= kFuseLds &&
               shape[ndim - 2] * n3 < (1LL << 31);       // row offsets in 32 bits
    }
}

int64_t mc_gaussian_mm_parts(int ndim, const int64_t *shape, const double *sigma, double truncate)
{
    std::vector<int> axes;
    bool fuse = false;
    gauss_axes(ndim, shape, sigma, truncate, axes, fuse);
    if (!fuse) return 0;
    int64_t nvox = 1;
    for (int i = 0; i < ndim; ++i) nvox *= shape[i];
    const int n2 = (int)shape[ndim - 2], n3 = (int)shape[ndim - 1];
    const int T2 = fuse_rows(n2, n3, gauss_radius(sigma[ndim - 2], truncate), gauss_radius(sigma[ndim - 1], truncate));
    return nvox / ((int64_t)n2 * n3) * ((n2 + T2 - 1) / T2);
}

mclahe_status mc_minmax_reduce(const float *src, int64_t n, float *dst, uint32_t m, hipStream_t st)
{
    if (m == 0) return MCLAHE_SUCCESS;
    hipLaunchKernelGGL(k_minmax_reduce, dim3(m), dim3(kT), 0, st, src, n, dst, m);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? MCLAHE_SUCCESS : mc_fail(MCLAHE_ERROR_HIP, "launch failed: %s", hipGetErrorString(e));
}

mclahe_status mc_gaussian_run(const void *d_in, int in_dtype, int ndim, const int64_t *shape, const double *sigma,
                              double truncate, float *d_out, void *d_workspace, size_t workspace_bytes, float *mm,
                              hipStream_t st)
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
    std::vector<int> axes;
    bool fuse = false;
    gauss_axes(ndim, shape, sigma, truncate, axes, fuse);
    const int P = (int)axes.size();
    if (P == 0) {
        const uint32_t blocks = (uint32_t)std::min<int64_t>(4096, (nvox + kT - 1) / kT);
        if (in_dtype == MCLAHE_U8) hipLaunchKernelGGL(k_to_float<uint8_t>, dim3(blocks), dim3(kT), 0, st, (const uint8_t *)d_in, d_out, nvox);
        else if (in_dtype == MCLAHE_U16) hipLaunchKernelGGL(k_to_float<uint16_t>, dim3(blocks), dim3(kT), 0, st, (const uint16_t *)d_in, d_out, nvox);
        else hipLaunchKernelGGL(k_to_float<float>, dim3(blocks), dim3(kT), 0, st, (const float *)d_in, d_out, nvox);
        const hipError_t e = hipGetLastError();
        return e == hipSuccess ? MCLAHE_SUCCESS : mc_fail(MCLAHE_ERROR_HIP, "launch failed: %s", hipGetErrorString(e));
    }
    // launches: one per smoothed axis, except that the last two axes go in
    // one fused pass when both are smoothed and the rows are short (that
    // pass also writes the min/max pairs when mm is given), and that two
    // consecutive smoothed axes before them, both strided, share one pass
    // (kind: 0 one axis, 1 the pair a, a + 1, 2 the last two axes)
    std::vector<std::pair<int, int>> groups;
    {
        const int Pn = fuse ? P - 2 : P;
        for (int k = 0; k < Pn;) {
            const int a = axes[k];
            if (k + 1 < Pn && axes[k + 1] == a + 1 && a + 1 < ndim - 1 &&
                pair_ok(gauss_radius(sigma[a], truncate), gauss_radius(sigma[a + 1], truncate))) {
                groups.push_back({a, 1});
                k += 2;
            } else {
                groups.push_back({a, 0});
                ++k;
            }
        }
        if (fuse) groups.push_back({ndim - 2, 2});
    }
    const int L = (int)groups.size();
    float *tmp = (float *)d_workspace;
    const float *src = nullptr;
    for (int k = 0; k < L; ++k) {
        const int a = groups[k].first, kind = groups[k].second;
        float *dst = ((L - 1 - k) % 2 == 0) ? d_out : tmp;   // the last launch lands in d_out
        Weights W;
        int r;
        gauss_weights(sigma[a], truncate, W, r);
        if (kind == 1) {
            Weights W1;
            int r1;
            gauss_weights(sigma[a + 1], truncate, W1, r1);
            int64_t S = 1;
            for (int i = a + 2; i < ndim; ++i) S *= shape[i];
            if (k == 0) {
                if (in_dtype == MCLAHE_U8) s = gauss_pair<uint8_t>((const uint8_t *)d_in, dst, nvox, shape[a], shape[a + 1], S, r, W, r1, W1, st);
                else if (in_dtype == MCLAHE_U16) s = gauss_pair<uint16_t>((const uint16_t *)d_in, dst, nvox, shape[a], shape[a + 1], S, r, W, r1, W1, st);
                else s = gauss_pair<float>((const float *)d_in, dst, nvox, shape[a], shape[a + 1], S, r, W, r1, W1, st);
            } else {
                s = gauss_pair<float>(src, dst, nvox, shape[a], shape[a + 1], S, r, W, r1, W1, st);
            }
        } else if (kind == 2) {
            Weights W3;
            int r3;
            gauss_weights(sigma[ndim - 1], truncate, W3, r3);
            const int n2 = (int)shape[ndim - 2], n3 = (int)shape[ndim - 1];
            if (k == 0) {
                if (in_dtype == MCLAHE_U8) s = gauss_last2<uint8_t>((const uint8_t *)d_in, dst, nvox, n2, n3, r, r3, W, W3, st, mm);
                else if (in_dtype == MCLAHE_U16) s = gauss_last2<uint16_t>((const uint16_t *)d_in, dst, nvox, n2, n3, r, r3, W, W3, st, mm);
                else s = gauss_last2<float>((const float *)d_in, dst, nvox, n2, n3, r, r3, W, W3, st, mm);
            } else {
                s = gauss_last2<float>(src, dst, nvox, n2, n3, r, r3, W, W3, st, mm);
            }
        } else {
            int64_t S = 1;
            for (int i = a + 1; i < ndim; ++i) S *= shape[i];
            if (k == 0) {
                if (in_dtype == MCLAHE_U8) s = gauss_pass<uint8_t>((const uint8_t *)d_in, dst, nvox, shape[a], S, r, W, st);
                else if (in_dtype == MCLAHE_U16) s = gauss_pass<uint16_t>((const uint16_t *)d_in, dst, nvox, shape[a], S, r, W, st);
                else s = gauss_pass<float>((const float *)d_in, dst, nvox, shape[a], S, r, W, st);
            } else {
                s = gauss_pass<float>(src, dst, nvox, shape[a], S, r, W, st);
            }
        }
        if (s) return s;
        src = dst;
    }
    return MCLAHE_SUCCESS;
}

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
    // (a fused last-two-axes pass needs no more: the bound stays one volume)
    *bytes = passes >= 2 ? ((sizeof(float) * nvox + 255) & ~size_t(255)) : 0;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_gaussian(const void *d_in, mclahe_dtype in_dtype, int ndim, const int64_t *shape,
                              const double *sigma, double truncate, float *d_out, void *d_workspace,
                              size_t workspace_bytes, void *hip_stream)
{
    return mc_gaussian_run(d_in, in_dtype, ndim, shape, sigma, truncate, d_out, d_workspace, workspace_bytes,
                           nullptr, (hipStream_t)hip_stream);
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
    for (int i = 0; i < g.N; ++i) {   // window value i: last axis fastest
        int q = i;
        int64_t off = 0;
        for (int a = ndim - 1; a >= 0; --a) {
            const int o = g.lo[a] + q % g.k[a];
            g.woff[i][a] = (int8_t)o;
            off += o * g.stride[a];
            q /= g.k[a];
        }
        g.off[i] = off;
    }
    const size_t esz = dtype == MCLAHE_U8 ? 1 : dtype == MCLAHE_U16 ? 2 : 4;
    const char *ib = (const char *)d_in, *ob = (const char *)d_out;
    if (ib < ob + esz * nvox && ob < ib + esz * nvox)
        return mc_fail(MCLAHE_ERROR_INVALID_VALUE, "input and output must not overlap");
    if ((nvox + kT - 1) / kT >= (1LL << 32)) return mc_fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large");
    g.slab_pre[0] = 0;
    for (int i = 0; i < ndim; ++i) {
        g.b0[i] = window[i] > 1 ? -g.lo[i] : 0;
        g.b1[i] = window[i] > 1 ? g.lo[i] + window[i] - 1 : 0;
        const int64_t cnt = std::min<int64_t>(g.b0[i] + g.b1[i], shape[i]);
        g.slab_pre[i + 1] = g.slab_pre[i] + cnt * (nvox / shape[i]);
    }
    hipStream_t hs = (hipStream_t)hip_stream;
    if (dtype == MCLAHE_U8) return median_launch<uint8_t>(d_in, d_out, g, hs);
    if (dtype == MCLAHE_U16) return median_launch<uint16_t>(d_in, d_out, g, hs);
    return median_launch<float>(d_in, d_out, g, hs);
}

}  // extern "C"
