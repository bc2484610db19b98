// gfx950 device code of the MCLAHE library.
//
// Every pass is written as a "work unit" device function that a work-group of
// MC_T = 256 threads (4 wave64s) executes.  The per-pass kernels launch one
// work-group per unit; the batched kernels launch one work-group per unit of
// every volume of a batch and call the very same functions, so both paths
// produce bit-identical results.
//
// Passes (Algorithm 1 of Stimper et al.; Sec. III.C-D):
//   range : global min/max (GHR) or per-kernel min/max (AHR)
//   hist  : per-kernel histograms over the virtually padded kernel grid
//   clip  : clip + equal redistribution (exact integers), inclusive CDF,
//           min-max normalisation -> per-kernel LUT
//   map   : 2^D-corner multilinear interpolation of the LUTs at every voxel
//
// Padding is never materialised.  A kernel's padded voxels mirror onto an
// interval ("box") of original coordinates per axis, hit once or twice
// (mc_kernel_box), so a histogram is accumulated over original voxels with
// integer weights equal to the product of the per-axis multiplicities.  This
// is exactly the count over the padded voxels, with each voxel read once.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "mc_desc.h"

namespace mc {

// ------------------------------------------------------------------ basics --
__device__ __forceinline__ int lane_id() { return threadIdx.x & 63; }

typedef float f4 __attribute__((ext_vector_type(4)));

// Touch every 64-byte line of a volume descriptor with loads issued
// together, before any field is used.  Fields are read where they are
// needed, many behind branches on others, and a launch's descriptor is in no
// cache yet (fresh kernel arguments, or a table just uploaded): without this
// the first read of each line waited for memory in turn, a chain of misses
// that dominated the duration of small launches.
__device__ __forceinline__ void warm_desc(const McVol &d)
{
    const char *p = reinterpret_cast<const char *>(&d);
    uint32_t acc = 0;
#pragma unroll
    for (int i = 0; i < (int)sizeof(McVol); i += 64) {
        uint32_t w;
        __builtin_memcpy(&w, p + i, sizeof w);
        acc ^= w;
    }
    asm volatile("; descriptor lines resident %0" ::"s"(acc));
}

// a / b for a >= 0 and b > 0 (b < 2^31).  The row counts and offsets a unit
// divides (one kernel column or cell box) nearly always fit 32 bits: a
// 32-bit division is a short instruction sequence, a 64-bit one a long one
// that dominated the set-up of small units, so the wide one runs only when
// a needs it.
__device__ __forceinline__ int64_t mc_div(int64_t a, int64_t b)
{
    if ((uint64_t)a <= 0xffffffffull && (uint64_t)b <= 0xffffffffull)
        return (int64_t)((uint32_t)a / (uint32_t)b);
    return a / b;
}

// Bin of v (single precision, no contraction; identical to the reading used
// by the oracle; scale = +inf for a degenerate range gives 0 / n-1 as well).
__device__ __forceinline__ int bin_of(float v, float lo, float scale, float nbf, int nbm1)
{
    (void)nbf;
    const float t = (v - lo) * scale;
    // v_cvt_u32_f32 truncates toward zero and saturates: t <= 0 and NaN give
    // 0, t >= 2^32 gives 2^32 - 1; the unsigned min then caps at n - 1.  So
    // !(t > 0) -> 0, t >= n -> n - 1, else (int)t, in two instructions.
    return (int)min(__float2uint_rz(t), (unsigned)nbm1);
}

__device__ __forceinline__ float range_scale(int nb, float lo, float hi)
{
    return __fdiv_rn((float)nb, hi - lo);
}

// Ordered integer image of a float for atomic min/max in LDS.
__device__ __forceinline__ int f2o(float f)
{
    const int i = __float_as_int(f);
    return i >= 0 ? i : i ^ 0x7fffffff;
}
__device__ __forceinline__ float o2f(int i) { return __int_as_float(i >= 0 ? i : i ^ 0x7fffffff); }

// V consecutive input elements as floats, with one 16- or 8-byte load.  A
// chunk starts at any element of a row (the HSA runtime runs the GPU in
// unaligned-access mode, so wide loads need no alignment); the last chunk
// of a row whose length is not a multiple of V is its last V elements.
template <typename Tin, int V>
__device__ __forceinline__ void load_chunk(const Tin *__restrict__ p, float (&f)[V])
{
    if constexpr (V == 1) {
        f[0] = (float)p[0];
    } else {
        constexpr int NW = V * (int)sizeof(Tin) / 4;   // 32-bit words: 4 or 2
        static_assert(NW == 4 || NW == 2, "a chunk is 16 or 8 bytes");
        uint32_t w[NW];
        if constexpr (NW == 4) {
            const uint4 q = *reinterpret_cast<const uint4 *>(p);
            w[0] = q.x;
            w[1] = q.y;
            w[2] = q.z;
            w[3] = q.w;
        } else {
            const uint2 q = *reinterpret_cast<const uint2 *>(p);
            w[0] = q.x;
            w[1] = q.y;
        }
        if constexpr (sizeof(Tin) == 4) {
#pragma unroll
            for (int i = 0; i < NW; ++i) f[i] = __uint_as_float(w[i]);
        } else if constexpr (sizeof(Tin) == 2) {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                f[2 * i] = (float)(w[i] & 0xffffu);
                f[2 * i + 1] = (float)(w[i] >> 16);
            }
        } else {
#pragma unroll
            for (int i = 0; i < NW; ++i) {
                f[4 * i] = (float)(w[i] & 0xffu);
                f[4 * i + 1] = (float)((w[i] >> 8) & 0xffu);
                f[4 * i + 2] = (float)((w[i] >> 16) & 0xffu);
                f[4 * i + 3] = (float)(w[i] >> 24);
            }
        }
    }
}

// Uniform copies of descriptor fields: scalar registers that the compiler
// keeps for a whole loop.  The batched kernels read their descriptor from
// device memory, and a field read inside a loop that stores to memory would
// otherwise be reloaded (with a vector load) on every iteration.
__device__ __forceinline__ int32_t mc_uniform(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
template <typename T>
__device__ __forceinline__ T *mc_uniform_ptr(T *p)
{
    const uint64_t v = (uint64_t)(uintptr_t)p;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (T *)(uintptr_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ McAxis mc_uniform_axis(const McAxis &a)
{
    McAxis r;
    r.s = mc_uniform(a.s);
    r.b = mc_uniform(a.b);
    r.p0 = mc_uniform(a.p0);
    r.p1 = mc_uniform(a.p1);
    r.n = mc_uniform(a.n);
    r.cw = mc_uniform(a.cw);
    return r;
}
__device__ __forceinline__ int64_t mc_uniform64(int64_t x)
{
    const uint64_t v = (uint64_t)x;
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
    return (int64_t)(((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ McBox mc_uniform_box(const McBox &b)
{
    return McBox{mc_uniform(b.lo), mc_uniform(b.hi), mc_uniform(b.olo), mc_uniform(b.ohi)};
}

__device__ __forceinline__ float load_elem(const void *in, int dt, int64_t i)
{
    if (dt == MC_U8) return (float)((const uint8_t *)in)[i];
    if (dt == MC_U16) return (float)((const uint16_t *)in)[i];
    return ((const float *)in)[i];
}

// The value an output element holds, as a float: y itself, or its integer
// code min(M, floor(y * M + 0.5)) for 8- and 16-bit output.
__device__ __forceinline__ float out_value(int dt, float y)
{
    if (dt == MC_F32) return y;
    const float M = dt == MC_U8 ? 255.0f : 65535.0f;
    const float q = floorf(y * M + 0.5f);
    return fminf(fmaxf(q, 0.0f), M);
}

// Quantised or float store of one output value.
__device__ __forceinline__ void store_elem(void *out, int dt, int64_t i, float y)
{
    const float q = out_value(dt, y);
    if (dt == MC_F32) ((float *)out)[i] = q;
    else if (dt == MC_U8) ((uint8_t *)out)[i] = (uint8_t)q;
    else ((uint16_t *)out)[i] = (uint16_t)q;
}

// Contrast-metric accumulators of one thread: minimum, maximum and float64
// sum of the input and of the stored output over the voxels it maps.
struct MetAcc {
    float mn[2], mx[2];
    double sum[2];
    __device__ __forceinline__ void init()
    {
        mn[0] = mn[1] = INFINITY;
        mx[0] = mx[1] = -INFINITY;
        sum[0] = sum[1] = 0.0;
    }
    __device__ __forceinline__ void add(float x, float y)
    {
        mn[0] = fminf(mn[0], x);
        mx[0] = fmaxf(mx[0], x);
        sum[0] += (double)x;
        mn[1] = fminf(mn[1], y);
        mx[1] = fmaxf(mx[1], y);
        sum[1] += (double)y;
    }
};

// Work-group reduction of the accumulators (NT threads; fixed order, so the
// partial is the same on every run) into the unit's record.  smem: at least
// 6 * 8 * (NT / 64) bytes, free for reuse (the caller has synchronised).
template <int NT>
__device__ __forceinline__ void met_flush(const MetAcc &a, char *smem, McMetPart *dst)
{
    constexpr int NW = NT / 64;
    float mn0 = a.mn[0], mx0 = a.mx[0], mn1 = a.mn[1], mx1 = a.mx[1];
    double s0 = a.sum[0], s1 = a.sum[1];
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn0 = fminf(mn0, __shfl_xor(mn0, o));
        mx0 = fmaxf(mx0, __shfl_xor(mx0, o));
        mn1 = fminf(mn1, __shfl_xor(mn1, o));
        mx1 = fmaxf(mx1, __shfl_xor(mx1, o));
        s0 += __shfl_xor(s0, o);
        s1 += __shfl_xor(s1, o);
    }
    float *f = (float *)smem;                  // [4][NW]
    double *g = (double *)(smem + 16 * NW);    // [2][NW]
    const int w = threadIdx.x >> 6;
    if (lane_id() == 0) {
        f[w] = mn0;
        f[NW + w] = mx0;
        f[2 * NW + w] = mn1;
        f[3 * NW + w] = mx1;
        g[w] = s0;
        g[NW + w] = s1;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        McMetPart r;
        r.mn[0] = f[0];
        r.mx[0] = f[NW];
        r.mn[1] = f[2 * NW];
        r.mx[1] = f[3 * NW];
        r.sum[0] = g[0];
        r.sum[1] = g[NW];
        for (int q = 1; q < NW; ++q) {
            r.mn[0] = fminf(r.mn[0], f[q]);
            r.mx[0] = fmaxf(r.mx[0], f[NW + q]);
            r.mn[1] = fminf(r.mn[1], f[2 * NW + q]);
            r.mx[1] = fmaxf(r.mx[1], f[3 * NW + q]);
            r.sum[0] += g[q];
            r.sum[1] += g[NW + q];
        }
        *dst = r;
    }
}

// Block-wide sum and exclusive scan over MC_T threads: wave-level shuffles
// within each wave64, then one pass over the per-wave totals in LDS scratch
// (at least MC_T / 64 words).  Integer sums: exact in any order.
__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o);
    return v;
}

__device__ __forceinline__ unsigned long long wave_incl_scan_u64(unsigned long long v)
{
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        const unsigned long long t = __shfl_up(v, o);
        if (lane >= o) v += t;
    }
    return v;
}

__device__ __forceinline__ unsigned long long block_sum_u64(unsigned long long v,
                                                            unsigned long long *s)
{
    constexpr int NW = MC_T / 64;
    v = wave_sum_u64(v);
    if (lane_id() == 0) s[threadIdx.x >> 6] = v;
    __syncthreads();
    unsigned long long r = 0;
#pragma unroll
    for (int w = 0; w < NW; ++w) r += s[w];
    __syncthreads();
    return r;
}

__device__ __forceinline__ unsigned long long block_exscan_u64(unsigned long long v,
                                                               unsigned long long *s)
{
    constexpr int NW = MC_T / 64;
    const int w = threadIdx.x >> 6;
    const unsigned long long inc = wave_incl_scan_u64(v);
    if (lane_id() == 63) s[w] = inc;
    __syncthreads();
    unsigned long long off = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) off += q < w ? s[q] : 0ull;
    __syncthreads();
    return off + inc - v;
}

// ----------------------------------------------------------- row iteration --
// A work unit covers a rectangular set of original voxels: an interval per
// outer axis (0..D-2) and a segment [xs, xe) of the last axis.  Its rows (one
// per outer coordinate tuple, last outer axis fastest) are split into
// contiguous chunks.  Row coordinates are kept as (o, r) with r the index on
// the innermost outer axis (D-2) and o the flattened index of axes 0..D-3,
// whose offset and weight come from an LDS table built once per unit.
struct RowSpace {
    int32_t lo[MC_MAXD], len[MC_MAXD];   // interval per outer axis
    int64_t rows;                         // product of len over outer axes
    int32_t in_lo, in_len;                // innermost outer axis (or dummy)
    int64_t in_stride;
};

__device__ __forceinline__ void rowspace_finish(const McVol &d, RowSpace &rs)
{
    const int D = d.D;
    rs.rows = 1;
    rs.in_lo = 0;
    rs.in_len = 1;
    rs.in_stride = 0;
#pragma unroll
    for (int i = 0; i < MC_MAXD - 1; ++i) {
        if (i < D - 1) rs.rows *= rs.len[i];
        if (i == D - 2) {
            rs.in_lo = rs.lo[i];
            rs.in_len = rs.len[i];
            rs.in_stride = d.stride[i];
        }
    }
}

__device__ __forceinline__ void mc_uniform_rows(RowSpace &rs)
{
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) {
        rs.lo[i] = mc_uniform(rs.lo[i]);
        rs.len[i] = mc_uniform(rs.len[i]);
    }
    rs.rows = mc_uniform64(rs.rows);
    rs.in_lo = mc_uniform(rs.in_lo);
    rs.in_len = mc_uniform(rs.in_len);
    rs.in_stride = mc_uniform64(rs.in_stride);
}

// Decode o (flattened axes 0..D-3) into coordinates; unrolled with guards so
// that every array index is a compile-time constant (no scratch memory).
__device__ __forceinline__ void decode_outer(const McVol &d, const RowSpace &rs, int64_t o64,
                                             int32_t (&x)[MC_MAXD])
{
    // o indexes the outer rows of one kernel or cell box: < 2^31
    const int D = d.D;
    uint32_t o = (uint32_t)o64;
#pragma unroll
    for (int i = MC_MAXD - 1; i >= 0; --i) {
        if (i <= D - 3) {
            const uint32_t q = o / (uint32_t)rs.len[i];
            x[i] = rs.lo[i] + (int32_t)(o - q * (uint32_t)rs.len[i]);
            o = q;
        }
    }
}

// Segment j of the last axis for the histogram / adaptive-range units:
// kernels [kA, kB) and original coordinates [xs, xe).
__device__ __forceinline__ void hist_segment(const McVol &d, int j, int &kA, int &kB, int &xs,
                                             int &xe)
{
    const McAxis &a = d.ax[d.D - 1];
    if (d.hP == 1) {
        kA = j * d.hG;
        kB = mc_min(kA + d.hG, a.n);
        xs = 0x7fffffff;
        xe = -1;
        for (int k = kA; k < kB; ++k) {
            const McBox b = mc_kernel_box(a, k);
            xs = mc_min(xs, b.lo);
            xe = mc_max(xe, b.hi);
        }
    } else {
        kA = j / d.hP;
        kB = kA + 1;
        const int pp = j - kA * d.hP;
        const McBox b = mc_kernel_box(a, kA);
        const int len = b.hi - b.lo;
        xs = b.lo + (int)mc_div((int64_t)len * pp, d.hP);
        xe = b.lo + (int)mc_div((int64_t)len * (pp + 1), d.hP);
    }
}

// Decode a histogram-unit index into its kernel column, segment and chunk,
// and the row space of the column.
__device__ __forceinline__ void hist_unit(const McVol &d, uint32_t wu, int64_t &col, int &seg,
                                          int &chunk, RowSpace &rs, McBox (&obox)[MC_MAXD],
                                          McBox &ib)
{
    ib = McBox{0, 1, 0, 0};
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) {
        obox[i] = McBox{0, 1, 0, 0};
        rs.lo[i] = 0;
        rs.len[i] = 1;
    }
    const int D = d.D;
    chunk = (int)(wu % (uint32_t)d.hCr);
    const uint32_t t1 = wu / (uint32_t)d.hCr;
    seg = (int)(t1 % (uint32_t)d.hS);
    col = (int64_t)(t1 / (uint32_t)d.hS);
    int64_t c = col;
#pragma unroll
    for (int i = MC_MAXD - 2; i >= 0; --i) {
        if (i <= D - 2) {
            const int64_t q = mc_div(c, d.ax[i].n);
            const int k = (int)(c - q * d.ax[i].n) + (i == 0 ? d.wk0 : 0);
            c = q;
            obox[i] = mc_kernel_box(d.ax[i], k);
            rs.lo[i] = obox[i].lo;
            rs.len[i] = obox[i].hi - obox[i].lo;
            if (i == D - 2) ib = obox[i];
        }
    }
    rowspace_finish(d, rs);
}

// Outer-row table for histogram units: element offset and integer weight of
// every o in [o0, o0 + cnt).
struct HistOTab {
    int64_t off;
    uint32_t w;
    uint32_t pad_;
};

__device__ __forceinline__ void build_hist_otab(const McVol &d, const RowSpace &rs,
                                                const McBox (&obox)[MC_MAXD], int64_t o0,
                                                int cnt, HistOTab *tab)
{
    const int D = d.D;
    // the strides, read once (scalar registers) rather than per entry
    int64_t st[MC_MAXD];
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) st[i] = i <= D - 3 ? mc_uniform64(d.stride[i]) : 0;
    for (int j = threadIdx.x; j < cnt; j += MC_T) {
        int32_t x[MC_MAXD];
        decode_outer(d, rs, o0 + j, x);
        int64_t off = 0;
        uint32_t w = 1;
#pragma unroll
        for (int i = 0; i < MC_MAXD; ++i) {
            if (i <= D - 3) {
                off += (int64_t)x[i] * st[i];
                w *= (uint32_t)mc_mult(obox[i], x[i]);
            }
        }
        tab[j].off = off;
        tab[j].w = w;
    }
}

// ------------------------------------------------------------ range (GHR) --
// Global min/max over the flat input.  Tiles of 4 * MC_T vectors are dealt to
// the units round-robin, so that the grid streams through the volume as one
// front rather than one contiguous block per unit (about 5 % faster on the
// 1 GiB volume); unit 0 also takes the vectors after the last whole tile.
template <typename Tin, int V>
__device__ void range_ghr_unit_v(const McVol &d, uint32_t u, float *red)
{
    const Tin *in = (const Tin *)d.in;
    const int64_t nvec = d.nvox / V;
    constexpr int64_t T = 4 * MC_T;
    const int64_t ntile = nvec / T;
    float mn = INFINITY, mx = -INFINITY;
    for (int64_t t = u; t < ntile; t += d.n_range_wu) {
        const int64_t i = t * T + threadIdx.x;
        float f[4][V];
#pragma unroll
        for (int k = 0; k < 4; ++k) load_chunk<Tin, V>(in + (i + k * MC_T) * V, f[k]);
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int e = 0; e < V; ++e) {
                mn = fminf(mn, f[k][e]);
                mx = fmaxf(mx, f[k][e]);
            }
    }
    if (u == 0) {
        for (int64_t i = ntile * T + threadIdx.x; i < nvec; i += MC_T) {
            float f[V];
            load_chunk<Tin, V>(in + i * V, f);
#pragma unroll
            for (int e = 0; e < V; ++e) {
                mn = fminf(mn, f[e]);
                mx = fmaxf(mx, f[e]);
            }
        }
    }
    if (u == d.n_range_wu - 1) {            // scalar tail of the last vector
        for (int64_t t = nvec * V + threadIdx.x; t < d.nvox; t += MC_T) {
            const float f = (float)in[t];
            mn = fminf(mn, f);
            mx = fmaxf(mx, f);
        }
    }
    red[threadIdx.x] = mn;
    red[MC_T + threadIdx.x] = mx;
    __syncthreads();
    for (int o = MC_T / 2; o > 0; o >>= 1) {
        if ((int)threadIdx.x < o) {
            red[threadIdx.x] = fminf(red[threadIdx.x], red[threadIdx.x + o]);
            red[MC_T + threadIdx.x] = fmaxf(red[MC_T + threadIdx.x], red[MC_T + threadIdx.x + o]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        d.rpart[2 * u] = red[0];
        d.rpart[2 * u + 1] = red[MC_T];
    }
}

template <typename Tin>
__device__ void range_ghr_unit(const McVol &d, uint32_t u, char *smem)
{
    constexpr int VM = mc_vec_elems((int)sizeof(Tin));
    // flat over the volume: vector loads need only an aligned base
    if (((uintptr_t)d.in & 15) == 0) range_ghr_unit_v<Tin, VM>(d, u, (float *)smem);
    else range_ghr_unit_v<Tin, 1>(d, u, (float *)smem);
}

// Work-group minimum and maximum (every thread gets both): butterfly
// shuffles inside each wave, then the MC_T / 64 wave results through LDS
// (ri: 2 MC_T / 64 ints).  Atomics of every lane to one LDS word were
// compiled into a loop over the active lanes, some 900 scalar instructions
// per wave, which dominated the set-up of a unit.  reuse: ri is written again
// later in the unit (a second barrier keeps that write after every read).
__device__ __forceinline__ void block_minmax_i32(int &mn, int &mx, int *ri, bool reuse = true)
{
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        mn = mc_min(mn, __shfl_xor(mn, o));
        mx = mc_max(mx, __shfl_xor(mx, o));
    }
    if (lane_id() == 0) {
        ri[2 * (threadIdx.x >> 6)] = mn;
        ri[2 * (threadIdx.x >> 6) + 1] = mx;
    }
    __syncthreads();
#pragma unroll
    for (int w = 0; w < MC_T / 64; ++w) {
        mn = mc_min(mn, ri[2 * w]);
        mx = mc_max(mx, ri[2 * w + 1]);
    }
    if (reuse) __syncthreads();
}

// Reduce the GHR partials (or take the user range); every unit that calls
// this gets the same lo, hi and scale.
__device__ __forceinline__ void ghr_range(const McVol &d, float *red, float &lo, float &hi,
                                          float &scale)
{
    if (d.has_user_range) {
        lo = d.user_lo;
        hi = d.user_hi;
    } else {
        // up to MC_STAGE partials per thread in flight at a time (a min and a
        // max: exact in any order)
        float mn = INFINITY, mx = -INFINITY;
        for (uint32_t i0 = threadIdx.x; i0 < d.n_range_wu; i0 += MC_STAGE * MC_T) {
            float2 pv[MC_STAGE];
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) {
                const uint32_t i = i0 + (uint32_t)q * MC_T;
                pv[q] = i < d.n_range_wu ? make_float2(d.rpart[2 * i], d.rpart[2 * i + 1])
                                         : make_float2(INFINITY, -INFINITY);
            }
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) {
                mn = fminf(mn, pv[q].x);
                mx = fmaxf(mx, pv[q].y);
            }
        }
        int imn = f2o(mn), imx = f2o(mx);
        block_minmax_i32(imn, imx, (int *)red);
        lo = o2f(imn);
        hi = o2f(imx);
    }
    scale = range_scale(d.nb, lo, hi);
}

// -------------------------------------------------- per-thread membership --
// For the V last-axis positions a thread owns inside a segment: the first
// kernel slot hit (or -1), its multiplicity, and any further (slot, mult)
// pairs packed in 'extra' (at most two more; only near folds of tiny axes).
template <int V>
struct Memb {
    int s1[V];
    uint32_t w1[V];
    uint32_t extra[V];
};

// Only three kernels can hold x: the one holding its padded position
// (x + p0) / b, kernel 0 if x is mirrored at the start (x < p0), and the
// last kernel if x is mirrored at the end (x >= s - p1): p0 and p1 are below
// b, so each fold lies inside one kernel.  They are visited in ascending
// order, as a scan of every kernel of the segment would find them.
template <int V>
__device__ __forceinline__ void build_memb(const McVol &d, int kA, int kB, int xs, int xe,
                                           int x0, Memb<V> &m)
{
    const McAxis &a = d.ax[d.D - 1];
    // While kernels are at least V wide, the padded positions of the V
    // elements fall in the kernel of the first one or the next: the boxes of
    // those two and of the two fold kernels serve every element (four boxes
    // per thread instead of up to three per element).
    const bool wide = a.b >= V;
    const int kd0 = (x0 + a.p0) / a.b;
    const McBox bfirst = mc_kernel_box(a, 0), blast = mc_kernel_box(a, a.n - 1);
    const McBox bd0 = mc_kernel_box(a, kd0), bd1 = mc_kernel_box(a, kd0 + 1);
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int x = x0 + e;
        m.s1[e] = -1;
        m.w1[e] = 0;
        m.extra[e] = 0;
        if (x < xs || x >= xe) continue;
        int kd;
        McBox bd;
        if (wide) {
            const bool up = x + a.p0 >= (kd0 + 1) * a.b;
            kd = up ? kd0 + 1 : kd0;
            bd = up ? bd1 : bd0;
        } else {
            kd = (x + a.p0) / a.b;
            bd = mc_kernel_box(a, kd);
        }
        int cand[3] = {x < a.p0 ? 0 : -1, kd, x >= a.s - a.p1 ? a.n - 1 : -1};
        if (cand[0] == kd) cand[0] = -1;          // the same kernel counts once
        if (cand[2] == kd) cand[2] = -1;
        const McBox *box[3] = {&bfirst, &bd, &blast};
        int found = 0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const int k = cand[c];
            if (k < kA || k >= kB) continue;
            const int w = mc_mult(*box[c], x);
            if (!w) continue;
            if (found == 0) {
                m.s1[e] = k - kA;
                m.w1[e] = (uint32_t)w;
            } else {
                m.extra[e] |= ((uint32_t)(k - kA + 1) | ((uint32_t)w << 8)) << (16 * (found - 1));
            }
            ++found;
        }
    }
}

// --------------------------------------------------- histogram / AHR range --
// LDS layout of a histogram unit.
struct HistLds {
    HistOTab *otab;     // [MC_OMAX]
    float *slot_lo;     // [hG]  (AHR)
    float *slot_sc;     // [hG]  (AHR)
    int *slot_mm;       // [hG][2] ordered min/max (AHR range pass)
    uint32_t *h;        // [hG][nb][R]
    float *red;         // [2*MC_T]
};

__device__ __forceinline__ HistLds hist_lds(const McVol &d, char *smem)
{
    HistLds L;
    char *p = smem;
    L.otab = (HistOTab *)p;
    p += sizeof(HistOTab) * MC_OMAX;
    L.red = (float *)p;
    p += sizeof(float) * 2 * MC_T;
    L.slot_lo = (float *)p;
    p += sizeof(float) * 64;
    L.slot_sc = (float *)p;
    p += sizeof(float) * 64;
    L.slot_mm = (int *)p;
    p += sizeof(int) * 128;
    L.h = (uint32_t *)p;
    return L;
}

// Wavefront-aggregated LDS histogram update: lanes whose key equals the
// first active lane's key add their summed weight with one atomic.
template <int PEEL>
__device__ __forceinline__ void hist_add(uint32_t *h, int key, uint32_t val, int cp)
{
    if constexpr (PEEL > 0) {
        unsigned long long act = __ballot(key >= 0);
#pragma unroll
        for (int r = 0; r < PEEL; ++r) {
            if (!act) break;
            // the leader index is wave-uniform: read its key and weight with
            // v_readlane (no LDS traffic, unlike a shuffle)
            const int leader = __ffsll((long long)act) - 1;
            const int lkey = __builtin_amdgcn_readlane(key, leader);
            const bool same = (key == lkey);
            const unsigned long long sm = __ballot(same);
            const uint32_t lval = (uint32_t)__builtin_amdgcn_readlane((int)val, leader);
            uint32_t sum;
            if (__ballot(same && val != lval) == 0ull) {
                sum = (uint32_t)__popcll(sm) * lval;
            } else {
                // weights are products of per-axis multiplicities (< 2^9):
                // add them bit plane by bit plane with ballots, which only
                // count active lanes
                sum = 0;
#pragma unroll
                for (int b = 0; b < 9; ++b)
                    sum += (uint32_t)__popcll(__ballot(same && ((val >> b) & 1u))) << b;
            }
            if (lane_id() == leader) atomicAdd(&h[lkey + cp], sum);
            if (same) key = -1;
            act &= ~sm;
        }
    }
    if (key >= 0) atomicAdd(&h[key + cp], val);
}

// VAL (uint8 input): the slots count values (256 per kernel) instead of
// bins; no range is needed here (the clip pass takes it and re-bins), and
// under a global range each unit also writes the smallest and largest value
// it counted.
template <typename Tin, int V, bool AHR, bool RANGE_ONLY, int PEEL, bool VAL = false, int UW = 4>
__device__ void hist_unit_v(const McVol &d, uint32_t wu, char *smem)
{
    static_assert(!VAL || (sizeof(Tin) == 1 && !RANGE_ONLY), "value slots: uint8 counting only");
    const int D = d.D, nb = VAL ? 256 : d.nb;
    HistLds L = hist_lds(d, smem);
    int64_t col;
    int seg, chunk;
    RowSpace rs;
    McBox obox[MC_MAXD], ib;
    hist_unit(d, wu, col, seg, chunk, rs, obox, ib);
    // the unit's geometry in scalar registers: kept, not recomputed from the
    // descriptor inside the loops
    mc_uniform_rows(rs);
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) obox[i] = mc_uniform_box(obox[i]);
    ib = mc_uniform_box(ib);
    int kA, kB, xs, xe;
    hist_segment(d, seg, kA, kB, xs, xe);
    const int nslot = kB - kA;
    const int R = RANGE_ONLY ? 1 : d.hR;
    // LDS words per slot: n*R + 1, odd, so that one bin of different slots
    // (kernels of the segment) falls in different banks
    const int SS = mc_hist_slot_stride(nb, R);

    // rows of this chunk
    const int64_t r0 = mc_div(rs.rows * chunk, d.hCr), r1 = mc_div(rs.rows * (chunk + 1), d.hCr);
    const int64_t o0 = mc_div(r0, rs.in_len);
    const int ocnt = r1 > r0 ? (int)(mc_div(r1 - 1, rs.in_len) - o0 + 1) : 0;
    build_hist_otab(d, rs, obox, o0, ocnt, L.otab);

    // global range (GHR) or this unit's kernels' ranges (AHR)
    float glo = 0.f, gsc = 0.f;
    const float nbf = (float)nb;
    const int nbm1 = nb - 1;
    if constexpr (!RANGE_ONLY) {
        if constexpr (VAL) {
            // values are counted as they are
        } else if constexpr (!AHR) {
            float ghi;
            ghr_range(d, L.red, glo, ghi, gsc);
            if (wu == 0 && threadIdx.x == 0) {
                d.range[0] = glo;
                d.range[1] = ghi;
                d.scale[0] = gsc;
            }
        } else {
            // kernel k's range: reduce the adaptive-range partials of every
            // unit covering k (all chunks; all parts when a kernel is split)
            const int64_t cb = col * d.hS;
            for (int s = threadIdx.x; s < nslot; s += MC_T) {
                const int k = kA + s;
                int sg0, nsg, sl;
                if (d.hP == 1) { sg0 = seg; nsg = 1; sl = s; }
                else { sg0 = k * d.hP; nsg = d.hP; sl = 0; }
                // MC_STAGE partials in flight at a time, reduced in the
                // order of the partials
                float mn = INFINITY, mx = -INFINITY;
                const int np = nsg * d.hCr;
                for (int p0 = 0; p0 < np; p0 += MC_STAGE) {
                    float2 pv[MC_STAGE];
#pragma unroll
                    for (int q = 0; q < MC_STAGE; ++q) {
                        const int pi = p0 + q;
                        pv[q] = make_float2(INFINITY, -INFINITY);
                        if (pi < np) {
                            const int g = pi / d.hCr, c = pi - g * d.hCr;
                            const int64_t u = (cb + sg0 + g) * d.hCr + c;
                            pv[q] = make_float2(d.rpart[(u * d.hG + sl) * 2], d.rpart[(u * d.hG + sl) * 2 + 1]);
                        }
                    }
#pragma unroll
                    for (int q = 0; q < MC_STAGE; ++q) {
                        mn = fminf(mn, pv[q].x);
                        mx = fmaxf(mx, pv[q].y);
                    }
                }
                L.slot_lo[s] = mn;
                L.slot_sc[s] = range_scale(nb, mn, mx);
                if (chunk == 0 && (d.hP == 1 || seg % d.hP == 0)) {
                    const int64_t kk = col * d.ax[D - 1].n + k;
                    d.range[2 * kk] = mn;
                    d.range[2 * kk + 1] = mx;
                    d.scale[kk] = L.slot_sc[s];
                }
            }
        }
        const int hsz = nslot * SS;
        for (int i = threadIdx.x; i < hsz; i += MC_T) L.h[i] = 0;
    } else {
        for (int i = threadIdx.x; i < 2 * nslot; i += MC_T)
            L.slot_mm[i] = (i & 1) ? f2o(-INFINITY) : f2o(INFINITY);
    }
    __syncthreads();

    // thread -> (chunk of the row segment, row within an iteration); a
    // split segment may be empty, then the unit only writes zero partials
    const int c_lo = xs / V, c_hi = xe > xs ? (xe + V - 1) / V : c_lo;
    const int cpr = c_hi - c_lo;
    const int rpi = cpr > 0 ? MC_T / cpr : 1;
    const int tch = cpr > 0 ? (int)threadIdx.x % cpr : 0;
    const int trow = cpr > 0 ? (int)threadIdx.x / cpr : MC_T;
    const bool tact = trow < rpi && r0 + trow < r1;
    // a chunk that would run past the row end (rows not a multiple of V) is
    // read as the row's last V elements instead; the ones it shares with the
    // previous chunk are skipped
    const int x0 = (c_lo + tch) * V, xl = mc_min(x0, d.ax[D - 1].s - V);
    Memb<V> m;
    build_memb<V>(d, kA, kB, mc_max(xs, x0), xe, xl, m);
    float lo1[V], sc1[V], mn[V], mx[V];
#pragma unroll
    for (int e = 0; e < V; ++e) {
        lo1[e] = glo;
        sc1[e] = gsc;
        if constexpr (AHR && !RANGE_ONLY && !VAL) {
            if (m.s1[e] >= 0) {
                lo1[e] = L.slot_lo[m.s1[e]];
                sc1[e] = L.slot_sc[m.s1[e]];
            }
        }
        mn[e] = INFINITY;
        mx[e] = -INFINITY;
    }
    const int cp = R > 1 ? (lane_id() & (R - 1)) : 0;
    // Per element, the byte offset of its first slot's replica in the LDS
    // histograms and its multiplicity; an element outside the segment adds
    // weight 0 to slot 0 instead of branching.  A bin then costs one shift
    // and add for its address and a 24-bit multiply for its weight.
    uint32_t hoff[V], w1[V];
    bool anyx = false;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        hoff[e] = m.s1[e] >= 0 ? (uint32_t)(m.s1[e] * SS + cp) * 4u : (uint32_t)cp * 4u;
        w1[e] = m.s1[e] >= 0 ? m.w1[e] : 0u;
        anyx = anyx || m.extra[e] != 0u;
    }
    const uint32_t bsh = 2u + (uint32_t)__builtin_ctz((unsigned)R);   // bin -> byte offset
    const Tin *in = (const Tin *)d.in;
    if (tact) {
        const int64_t rstart = r0 + trow;
        int64_t o = mc_div(rstart, rs.in_len);
        int r = (int)(rstart - o * rs.in_len);
        const int64_t so = mc_div(rpi, rs.in_len);
        const int sr = (int)(rpi - so * rs.in_len);
        const int64_t xoff = xl;
        // U rows per step.  Software pipelined: the loads of the next U rows
        // are issued before the current U rows are binned, so every wave
        // keeps up to 2U wide loads in flight while it works.  UW: rows per
        // step of 16-byte chunks (4 for a volume alone; batched launches take
        // 2, which needs 77 instead of 111 VGPRs, six waves per SIMD instead
        // of four: faster on the many small units of a batch, slower on the
        // large ones of a volume alone)
        constexpr int U = V >= 8 ? 2 : UW;
        auto prep_load = [&](int64_t rw, uint32_t (&wr)[U], bool (&okk)[U], float (&fl)[U][V]) {
            int64_t offs[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                okk[u] = rw + (int64_t)u * rpi < r1;
                const HistOTab te = L.otab[okk[u] ? (int)(o - o0) : 0];
                const int xin = rs.in_lo + r;
                offs[u] = te.off + (int64_t)xin * rs.in_stride + xoff;
                wr[u] = te.w * (uint32_t)mc_mult(ib, xin);
                r += sr;
                o += so;
                if (r >= rs.in_len) {
                    r -= rs.in_len;
                    o += 1;
                }
            }
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (okk[u]) load_chunk<Tin, V>(in + offs[u], fl[u]);
        };
        // XT: whether this wave has elements with further memberships (a
        // wave-uniform value, so the loop without them is a separate copy
        // that tests nothing per element)
        auto process = [&](auto XT, int64_t rw, const uint32_t (&wr)[U], const bool (&okk)[U],
                           const float (&fl)[U][V]) {
            constexpr bool XW = decltype(XT)::value;
#pragma unroll
            for (int u = 0; u < U; ++u) {
            if (!okk[u]) break;
            const float (&f)[V] = fl[u];
            const uint32_t wrow = wr[u];
            if constexpr (!RANGE_ONLY && PEEL == 0) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const uint32_t b = VAL ? (uint32_t)f[e] : (uint32_t)bin_of(f[e], lo1[e], sc1[e], nbf, nbm1);
                    atomicAdd((uint32_t *)((char *)L.h + ((b << bsh) + hoff[e])), __umul24(wrow, w1[e]));
                }
            }
            // LDS word of (slot, bin) per element (replica 0; -1: no update)
            // and its weight (wavefront aggregation only)
            int key[V];
            uint32_t wk[V];
            if constexpr (!RANGE_ONLY && PEEL > 0) {
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    key[e] = -1;
                    wk[e] = wrow * m.w1[e];
                    if (m.s1[e] >= 0) {
                        key[e] = m.s1[e] * SS + (VAL ? (int)f[e] : bin_of(f[e], lo1[e], sc1[e], nbf, nbm1)) * R;
                    }
                }
            }
            // the further memberships of elements near a fold
            if constexpr (RANGE_ONLY || PEEL > 0 || XW) {
#pragma unroll
            for (int e = 0; e < V; ++e) {
                if constexpr (RANGE_ONLY) {
                    mn[e] = fminf(mn[e], f[e]);
                    mx[e] = fmaxf(mx[e], f[e]);
                    if (m.extra[e]) {
                        uint32_t ex = m.extra[e];
                        while (ex) {
                            const int s = (int)(ex & 0xff) - 1;
                            atomicMin(&L.slot_mm[2 * s], f2o(f[e]));
                            atomicMax(&L.slot_mm[2 * s + 1], f2o(f[e]));
                            ex >>= 16;
                        }
                    }
                } else {
                    if constexpr (PEEL > 0) hist_add<PEEL>(L.h, key[e], wk[e], cp);
                    if (m.extra[e]) {
                        uint32_t ex = m.extra[e];
                        while (ex) {
                            const int s = (int)(ex & 0xff) - 1;
                            const uint32_t w = (ex >> 8) & 0xff;
                            const float lo = AHR && !VAL ? L.slot_lo[s] : glo;
                            const float sc = AHR && !VAL ? L.slot_sc[s] : gsc;
                            const int b = VAL ? (int)f[e] : bin_of(f[e], lo, sc, nbf, nbm1);
                            atomicAdd(&L.h[s * SS + b * R + cp], wrow * w);
                            ex >>= 16;
                        }
                    }
                }
            }
            }
            }
        };
        auto rows = [&](auto XT) {
            uint32_t wA[U], wB[U];
            bool okA[U], okB[U];
            float fA[U][V], fB[U][V];
            const int64_t step = (int64_t)U * rpi;
            int64_t row = rstart;
            prep_load(row, wA, okA, fA);
            for (;;) {
                const int64_t nb = row + step;
                if (nb < r1) prep_load(nb, wB, okB, fB);
                process(XT, row, wA, okA, fA);
                row = nb;
                if (row >= r1) break;
                const int64_t na = row + step;
                if (na < r1) prep_load(na, wA, okA, fA);
                process(XT, row, wB, okB, fB);
                row = na;
                if (row >= r1) break;
            }
        };
        if constexpr (RANGE_ONLY || PEEL > 0) {
            rows(std::true_type{});
        } else {
            if (__any(anyx ? 1 : 0)) rows(std::true_type{});
            else rows(std::false_type{});
        }
    }
    if constexpr (RANGE_ONLY) {
#pragma unroll
        for (int e = 0; e < V; ++e) {
            if (m.s1[e] >= 0 && mn[e] <= mx[e]) {
                atomicMin(&L.slot_mm[2 * m.s1[e]], f2o(mn[e]));
                atomicMax(&L.slot_mm[2 * m.s1[e] + 1], f2o(mx[e]));
            }
        }
    }
    __syncthreads();
    if constexpr (RANGE_ONLY) {
        for (int s = threadIdx.x; s < d.hG; s += MC_T) {
            float a = INFINITY, b = -INFINITY;
            if (s < nslot) {
                a = o2f(L.slot_mm[2 * s]);
                b = o2f(L.slot_mm[2 * s + 1]);
            }
            d.rpart[((int64_t)wu * d.hG + s) * 2] = a;
            d.rpart[((int64_t)wu * d.hG + s) * 2 + 1] = b;
        }
    } else {
        // flush: partial histogram of every slot (replicas summed)
        uint32_t *dst = d.part + (int64_t)wu * d.hG * nb;
        const int tot = d.hG * nb;
        int vmin = 256, vmax = -1;   // VAL: smallest and largest value counted
        for (int i = threadIdx.x; i < tot; i += MC_T) {
            uint32_t s = 0;
            if (i < nslot * nb) {
                const int sl = i / nb, b = i - sl * nb;
                for (int c = 0; c < R; ++c) s += L.h[sl * SS + b * R + c];
                if (VAL && s) {
                    vmin = mc_min(vmin, b);
                    vmax = mc_max(vmax, b);
                }
            }
            dst[i] = s;
        }
        if constexpr (VAL && !AHR) {
            // the unit's (min, max) value, for the global range of the clip
            // pass (+inf/-inf when the unit counted nothing)
            block_minmax_i32(vmin, vmax, (int *)L.red, false);   // the unit's last use of LDS
            if (threadIdx.x == 0) {
                d.rpart[2 * (int64_t)wu] = vmax >= 0 ? (float)vmin : INFINITY;
                d.rpart[2 * (int64_t)wu + 1] = vmax >= 0 ? (float)vmax : -INFINITY;
            }
        }
    }
}

// VAL: value slots (uint8 input with d.vhist set), a kernel of its own so
// that each variant gets the registers it needs
template <typename Tin, bool AHR, bool RANGE_ONLY, int PEEL, bool VAL = false, int UW = 4>
__device__ void hist_unit_dispatch(const McVol &d, uint32_t wu, char *smem)
{
    constexpr int VM = mc_vec_elems((int)sizeof(Tin));
    if (d.vec == VM) hist_unit_v<Tin, VM, AHR, RANGE_ONLY, PEEL, VAL, UW>(d, wu, smem);
    else hist_unit_v<Tin, 1, AHR, RANGE_ONLY, PEEL, VAL, UW>(d, wu, smem);
}

// ----------------------------------------------------- clip + CDF + LUT --
// One unit per kernel: sum the partial histograms, clip at C and share the
// excess equally (H = n*min(h,C) + E, exact), inclusive CDF, normalised LUT.
// Comparison variants (d.redist): the equal sharing repeated while an excess
// remains, at most d.rounds rounds, round r in units of 1/n^r (the clip level
// becomes C n^r); or integer counts, floor(E/n) to every bin and the
// remainder R one each to bins 0, s, 2s, .. (s = max(n/R, 1)).  Their H goes
// through the clipped array, which each thread reads back for its own bins.
__device__ __forceinline__ void clip_variant(const McVol &d, uint32_t k, const uint32_t *hk, int j0, int j1,
                                          unsigned long long C, unsigned long long E, unsigned long long *s64)
{
    const int nb = d.nb;
    const unsigned long long nbu = (unsigned long long)nb;
    unsigned long long *Hk = d.clipped + (int64_t)k * nb;
    unsigned long long tsum = 0;
    if (d.redist == MC_REDIST_INTEGER) {
        const unsigned long long q = E / nbu, R = E - q * nbu;
        const unsigned long long st = R ? (nbu / R > 1 ? nbu / R : 1ull) : 1ull;
        for (int j = j0; j < j1; ++j) {
            const unsigned long long h = hk[j], ju = (unsigned long long)j;
            const unsigned long long H = (h < C ? h : C) + q + ((R && ju % st == 0 && ju / st < R) ? 1ull : 0ull);
            Hk[j] = H;
            tsum += H;
        }
    } else {
        for (int j = j0; j < j1; ++j) {
            const unsigned long long h = hk[j];
            Hk[j] = nbu * (h < C ? h : C) + E;
        }
        unsigned long long Cr = C * nbu;
        for (int r = 2; r <= d.rounds; ++r) {
            unsigned long long ex = 0;
            for (int j = j0; j < j1; ++j) ex += Hk[j] > Cr ? Hk[j] - Cr : 0ull;
            const unsigned long long Er = block_sum_u64(ex, s64);
            if (Er == 0) break;                 // block-uniform
            for (int j = j0; j < j1; ++j) Hk[j] = nbu * (Hk[j] < Cr ? Hk[j] : Cr) + Er;
            Cr *= nbu;
        }
        for (int j = j0; j < j1; ++j) tsum += Hk[j];
    }
    const unsigned long long pre = block_exscan_u64(tsum, s64);
    if (threadIdx.x == MC_T - 1) s64[0] = pre + tsum;
    if (threadIdx.x == 0) s64[1] = Hk[0];       // bin 0 is thread 0's own
    __syncthreads();
    const unsigned long long total = s64[0], c0 = s64[1];
    const unsigned long long den = total - c0;
    unsigned long long acc = pre;
    float *lk = d.lut + (int64_t)k * nb;
    for (int j = j0; j < j1; ++j) {
        acc += Hk[j];
        const double m = den == 0 ? (double)j / (double)(nb - 1) : (double)(acc - c0) / (double)den;
        lk[j] = (float)m;
    }
}

__device__ void clip_unit(const McVol &d, uint32_t k, char *smem)
{
    unsigned long long *s64 = (unsigned long long *)smem;
    const int nb = d.nb;
    const int nl = d.ax[d.D - 1].n;
    const int64_t col = mc_div((int64_t)k, nl);
    const int kl = (int)(k - col * nl);
    int sg0, nsg, sl;
    if (d.hP == 1) { sg0 = kl / d.hG; nsg = 1; sl = kl - sg0 * d.hG; }
    else { sg0 = kl * d.hP; nsg = d.hP; sl = 0; }
    const int per = (nb + MC_T - 1) / MC_T;
    const int j0 = mc_min(nb, (int)threadIdx.x * per), j1 = mc_min(nb, j0 + per);
    const unsigned long long C = (unsigned long long)d.clipC;
    uint32_t *hk = d.hist + (int64_t)k * nb;
    unsigned long long smin = 0, exc = 0;
    const int np = nsg * d.hCr;   // partials of this kernel
    uint32_t *hs = (uint32_t *)(smem + MC_T * 8);   // counted values re-binned (vhist)
    if (d.vhist) {
        // uint8 input counted per value: thread v sums the kernel's count of
        // value v, the range is taken (per kernel, the caller's, or the
        // smallest and largest value any unit counted), and the values are
        // re-binned exactly as the histogram pass bins a voxel of that value.
        // The first range partials and the counts are all in flight before
        // either is reduced.
        const int v = threadIdx.x;   // MC_T == 256 values
        const bool gpart = d.mode == MC_GHR && !d.has_user_range;
        float2 rv[MC_STAGE];
#pragma unroll
        for (int q = 0; q < MC_STAGE; ++q) {
            const uint32_t i = (uint32_t)threadIdx.x + (uint32_t)q * MC_T;
            rv[q] = gpart && i < d.n_hist_wu ? make_float2(d.rpart[2 * (int64_t)i], d.rpart[2 * (int64_t)i + 1])
                                             : make_float2(INFINITY, -INFINITY);
        }
        uint32_t cnt = 0;
        for (int p0 = 0; p0 < np; p0 += MC_STAGE) {
            uint32_t pv[MC_STAGE];
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) {
                const int pi = p0 + q;
                pv[q] = 0u;
                if (pi < np) {
                    const int g = pi / d.hCr, c = pi - g * d.hCr;
                    const int64_t u = (col * d.hS + sg0 + g) * d.hCr + c;
                    pv[q] = d.part[(u * d.hG + sl) * 256 + v];
                }
            }
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) cnt += pv[q];
        }
        float lo, hi;
        if (d.mode == MC_GHR && d.has_user_range) {
            lo = d.user_lo;
            hi = d.user_hi;
        } else {
            // order-preserving integers
            int mn = 0x7fffffff, mx = (int)0x80000000;
            if (d.mode == MC_AHR) {
                if (cnt) mn = mx = f2o((float)v);
            } else {
#pragma unroll
                for (int q = 0; q < MC_STAGE; ++q) {
                    mn = mc_min(mn, f2o(rv[q].x));
                    mx = mc_max(mx, f2o(rv[q].y));
                }
                for (uint32_t i0 = threadIdx.x + MC_STAGE * MC_T; i0 < d.n_hist_wu; i0 += MC_STAGE * MC_T) {
#pragma unroll
                    for (int q = 0; q < MC_STAGE; ++q) {
                        const uint32_t i = i0 + (uint32_t)q * MC_T;
                        rv[q] = i < d.n_hist_wu ? make_float2(d.rpart[2 * (int64_t)i], d.rpart[2 * (int64_t)i + 1])
                                                : make_float2(INFINITY, -INFINITY);
                    }
#pragma unroll
                    for (int q = 0; q < MC_STAGE; ++q) {
                        mn = mc_min(mn, f2o(rv[q].x));
                        mx = mc_max(mx, f2o(rv[q].y));
                    }
                }
            }
            for (int i = threadIdx.x; i < nb; i += MC_T) hs[i] = 0u;
            block_minmax_i32(mn, mx, (int *)smem, false);   // its barrier also orders the zeroing
            lo = o2f(mn);
            hi = o2f(mx);
        }
        const float sc = range_scale(nb, lo, hi);
        if (threadIdx.x == 0) {
            if (d.mode == MC_AHR) {
                d.range[2 * (int64_t)k] = lo;
                d.range[2 * (int64_t)k + 1] = hi;
                d.scale[k] = sc;
            } else if (k == 0) {
                d.range[0] = lo;
                d.range[1] = hi;
                d.scale[0] = sc;
            }
        }
        if (d.mode == MC_GHR && d.has_user_range) {
            for (int i = threadIdx.x; i < nb; i += MC_T) hs[i] = 0u;
            __syncthreads();
        }
        if (cnt) atomicAdd(&hs[bin_of((float)v, lo, sc, (float)nb, nb - 1)], cnt);
        __syncthreads();
    }
    for (int j = j0; j < j1; ++j) {
        // MC_STAGE partials in flight at a time (integer sums: exact in any order)
        uint32_t h = d.vhist ? hs[j] : 0u;
        for (int p0 = 0; p0 < (d.vhist ? 0 : np); p0 += MC_STAGE) {
            uint32_t pv[MC_STAGE];
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) {
                const int pi = p0 + q;
                pv[q] = 0u;
                if (pi < np) {
                    const int g = pi / d.hCr, c = pi - g * d.hCr;
                    const int64_t u = (col * d.hS + sg0 + g) * d.hCr + c;
                    pv[q] = d.part[(u * d.hG + sl) * nb + j];
                }
            }
#pragma unroll
            for (int q = 0; q < MC_STAGE; ++q) h += pv[q];
        }
        hk[j] = h;
        smin += h < C ? h : C;
        exc += h > C ? h - C : 0ull;
    }
    // One block pass with one barrier: the sum of min(h, C) over the bins
    // of the threads before this one (wave scans, then the wave totals
    // through LDS), the block totals of min(h, C) and of the excess E, and
    // bin 0's min(h, C).  With H_j = n min(h_j, C) + E, the prefix of H
    // before bin j0, H_0 and the total of H follow in exact integers (the
    // bins are dealt to the threads in order, j0 of them before this one).
    constexpr int NW = MC_T / 64;
    const int w = (int)(threadIdx.x >> 6);
    const unsigned long long sinc = wave_incl_scan_u64(smin);
    const unsigned long long esum = wave_sum_u64(exc);
    if (lane_id() == 63) s64[w] = sinc;
    if (lane_id() == 0) s64[NW + w] = esum;
    if (threadIdx.x == 0) {
        const uint32_t h0 = hk[0];   // bin 0 is thread 0's own
        s64[2 * NW] = h0 < C ? h0 : C;
    }
    __syncthreads();
    unsigned long long spre = sinc - smin, stot = 0, E = 0;
#pragma unroll
    for (int q = 0; q < NW; ++q) {
        stot += s64[q];
        spre += q < w ? s64[q] : 0ull;
        E += s64[NW + q];
    }
    const unsigned long long m0 = s64[2 * NW];
    const unsigned long long nbu = (unsigned long long)nb;
    if (d.redist != MC_REDIST_EQUAL) {
        __syncthreads();   // every thread has read the exchange before it is reused
        clip_variant(d, k, hk, j0, j1, C, E, s64);
        return;
    }
    // c0 = H_0, total = sum H (= n*K); both block-uniform
    const unsigned long long total = nbu * stot + nbu * E, c0 = nbu * m0 + E;
    const unsigned long long den = total - c0;
    unsigned long long acc = nbu * spre + (unsigned long long)j0 * E;
    unsigned long long *Hk = d.clipped + (int64_t)k * nb;
    float *lk = d.lut + (int64_t)k * nb;
    for (int j = j0; j < j1; ++j) {
        const uint32_t h = hk[j];
        const unsigned long long H = nbu * (h < C ? h : C) + E;
        acc += H;
        Hk[j] = H;
        const double m = den == 0 ? (double)j / (double)(nb - 1)
                                  : (double)(acc - c0) / (double)den;
        lk[j] = (float)m;
    }
}

// ------------------------------------------------------------------- map --
// Interpolation units (MC_MAP_T threads): a cell column (one cell per outer
// axis) x a group of cells on the last axis x a chunk of rows.  The LUTs of the 2^(D-1) outer
// corner kernels times the group's last-axis kernels are staged in LDS.
// Work-groups are dispatched to the 8 XCDs of the chip round-robin, and each
// XCD has its own L2.  The mS units that share the same rows (one per
// last-axis group) read the same cache lines, so they are ordered to run
// back to back on one XCD: unit index u on XCD u % 8 takes the k-th unit of
// that XCD, k = u / 8, as group k % mS of row set (k / mS) * 8 + u % 8.
// Only the order changes, never what a unit computes.
__device__ __forceinline__ uint32_t map_unit_order(const McVol &d, uint32_t u)
{
    const uint32_t ns = (uint32_t)d.mS;
    const uint32_t ncc = d.n_map_wu / ns;           // (cell column, unit chunk) pairs
    if (ns == 1 || (ncc & 7u)) return u;
    const uint32_t x = u & 7u, k = u >> 3;
    const uint32_t g = k % ns, cc = (k / ns) * 8u + x;
    const uint32_t col = cc / (uint32_t)d.mU, chunk = cc - col * (uint32_t)d.mU;
    return (col * ns + g) * (uint32_t)d.mU + chunk;
}

__device__ __forceinline__ void map_unit_decode(const McVol &d, uint32_t wu, int &chunk, int &grp,
                                                int32_t (&cidx)[MC_MAXD], RowSpace &rs)
{
    const int D = d.D;
    wu = map_unit_order(d, wu);
    chunk = (int)(wu % (uint32_t)d.mU);      // unit chunk: row chunks [chunk*mK, +mK)
    const uint32_t t1 = wu / (uint32_t)d.mU;
    grp = (int)(t1 % (uint32_t)d.mS);
    int64_t c = (int64_t)(t1 / (uint32_t)d.mS);
#pragma unroll
    for (int i = MC_MAXD - 2; i >= 0; --i) {
        if (i <= D - 2) {
            const int nc = d.ax[i].n - 1;
            const int64_t q = mc_div(c, nc);
            cidx[i] = (int)(c - q * nc) + (i == 0 ? d.wc0 : 0);
            c = q;
            int lo, hi;
            mc_cell_range(d.ax[i], cidx[i], lo, hi);
            rs.lo[i] = lo;
            rs.len[i] = hi - lo;
        }
    }
    rowspace_finish(d, rs);
}

// Weight of x towards the upper kernel of its cell c along axis a,
// m / (2b) as m times the single-precision reciprocal of 2b (exact for
// power-of-two b, otherwise within one ulp; the same expression is used by
// every kernel, so plain and batched results stay bit-identical).
__device__ __forceinline__ float cell_weight(const McAxis &a, int c, int x)
{
    return (float)mc_cell_m(a, c, x) * (1.0f / (float)(2 * a.b));
}

template <int D>
struct MapOTab {
    static constexpr int NOH = D >= 3 ? (1 << (D - 2)) : 1;
    int64_t off;
    float coef[NOH];
};

// NT: work-group size (the per-pass kernels use mc_map_threads(AHR); the
// persistent batched kernel runs every unit with MC_T threads)
template <typename Tin, int D, bool AHR, int V, bool MET, int NT>
__device__ void map_unit_v(const McVol &d, uint32_t wu, char *smem)
{
    constexpr int NC = 1 << D;                 // corners
    constexpr int NO = 1 << (D - 1);           // outer corners
    using OT = MapOTab<D>;
    constexpr int NOH = OT::NOH;
    const int nb = d.nb;
    int chunk, grp;
    int32_t cidx[MC_MAXD];
    RowSpace rs;
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) {
        cidx[i] = 0;
        rs.lo[i] = 0;
        rs.len[i] = 1;
    }
    map_unit_decode(d, wu, chunk, grp, cidx, rs);
    // the unit's geometry, and the outer axes and strides of its row table,
    // in scalar registers (read once, not per table entry)
    mc_uniform_rows(rs);
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) cidx[i] = mc_uniform(cidx[i]);
    McAxis oax[MC_MAXD];
    int64_t ost[MC_MAXD];
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) {
        oax[i] = i < D - 2 ? mc_uniform_axis(d.ax[i]) : McAxis{1, 1, 0, 0, 1, 0};
        ost[i] = i < D - 2 ? mc_uniform64(d.stride[i]) : 0;
    }
    const McAxis &al = d.ax[D - 1];
    int cA, cB, xs, xe, tmp;
    if (d.mP == 1) {
        cA = grp * d.mG;
        cB = mc_min(cA + d.mG, al.n - 1);
        mc_cell_range(al, cA, xs, tmp);
        mc_cell_range(al, cB - 1, tmp, xe);
    } else {   // part (grp % mP) of cell (grp / mP)
        cA = grp / d.mP;
        cB = cA + 1;
        const int pp = grp - cA * d.mP;
        int lo, hi;
        mc_cell_range(al, cA, lo, hi);
        xs = lo + (int)mc_div((int64_t)(hi - lo) * pp, d.mP);
        xe = lo + (int)mc_div((int64_t)(hi - lo) * (pp + 1), d.mP);
    }
    const int ncl = cB - cA;

    OT *otab = (OT *)smem;
    float *lut = (float *)(smem + sizeof(OT) * MC_OMAX);

    // kernel-grid strides (last axis fastest)
    int64_t kst[MC_MAXD];
    {
        int64_t s = 1;
#pragma unroll
        for (int i = D - 1; i >= 0; --i) {
            kst[i] = s;
            s *= d.ax[i].n;
        }
    }
    int64_t kbase = 0;   // kernel index of outer corner 0, last-axis kernel 0
#pragma unroll
    for (int i = 0; i < D - 1; ++i) kbase += (int64_t)cidx[i] * kst[i];

    // stage LUTs.  GHR: one row of SB floats per bin holding [lk][corner'],
    // SB padded to an odd number of LDS read units so that lanes reading
    // different bins spread over the banks.  AHR: [lk*NO + corner'][bin].
    const int nlk = ncl + 1;
    const int SB = AHR ? 0 : mc_lut_stride(nlk, NO);
    {
        // every thread issues up to MC_STAGE loads before its first LDS
        // store: one kernel's LUT per step would wait for memory once per
        // staged kernel (2^(D-1) (mG + 1) of them), a fixed latency that
        // dominated units of a few hundred thousand voxels
        constexpr int ST = MC_STAGE;
        const int tot = nlk * NO * nb;
        for (int i0 = threadIdx.x; i0 < tot; i0 += ST * NT) {
            float val[ST];
            int dst[ST];
#pragma unroll
            for (int q = 0; q < ST; ++q) {
                const int i = i0 + q * NT;
                dst[q] = -1;
                val[q] = 0.f;
                if (i < tot) {
                    const int t = i / nb, b = i - t * nb;
                    const int co = t % NO, lk = t / NO;   // NO is a power of two
                    int64_t kid = kbase + cA + lk;
#pragma unroll
                    for (int j = 0; j < D - 1; ++j)
                        if ((co >> (D - 2 - j)) & 1) kid += kst[j];
                    val[q] = d.lut[kid * nb + b];
                    dst[q] = AHR ? i : __umul24(b, SB) + lk * NO + co;
                }
            }
#pragma unroll
            for (int q = 0; q < ST; ++q)
                if (dst[q] >= 0) lut[dst[q]] = val[q];
        }
    }
    // per-corner ranges (AHR: one last-axis cell per unit)
    float clo[NC], csc[NC];
    float glo = 0.f, gsc = 0.f;
    if constexpr (AHR) {
#pragma unroll
        for (int c = 0; c < NC; ++c) {
            const int lk = c / NO, co = c % NO;
            int64_t kid = kbase + cA + lk;
#pragma unroll
            for (int j = 0; j < D - 1; ++j)
                if ((co >> (D - 2 - j)) & 1) kid += kst[j];
            clo[c] = d.range[2 * kid];
            csc[c] = d.scale[kid];
        }
    } else {
        glo = d.range[0];
        gsc = d.scale[0];
#pragma unroll
        for (int c = 0; c < NC; ++c) clo[c] = csc[c] = 0.f;
    }

    // the LUTs (and AHR ranges) staged above are published by the first
    // chunk's barrier below
    if (xe <= xs) {         // an empty split part (uniform over the work-group)
        if constexpr (MET) {
            if (threadIdx.x == 0) d.met[wu] = McMetPart{{INFINITY, INFINITY}, {-INFINITY, -INFINITY}, {0.0, 0.0}};
        }
        return;
    }
    MetAcc macc;
    if constexpr (MET) macc.init();
    // thread mapping along the last axis (a split cell part may be empty)
    const int c_lo = xs / V, c_hi = (xe + V - 1) / V;
    const int cpr = c_hi - c_lo;
    const int rpi = NT / cpr;
    const int tch = threadIdx.x % cpr, trow = threadIdx.x / cpr;
    const bool tact = trow < rpi;
    // a chunk that would run past the row end (rows not a multiple of V) is
    // read as the row's last V elements instead; the ones it shares with the
    // previous chunk are skipped
    const int x0 = (c_lo + tch) * V;
    const int64_t xoff = mc_min(x0, al.s - V);
    const int xvs = mc_max(xs, x0);   // first position this thread maps
    int lbase[V];      // LDS offset of the voxel's last-axis kernel pair
    float wl[V];
    bool val[V];
    bool allv = true;
#pragma unroll
    for (int e = 0; e < V; ++e) {
        const int x = (int)xoff + e;
        val[e] = x >= xvs && x < xe;
        allv = allv && val[e];
        int c = cA;
        if (val[e]) {
            // cell of x on the last axis: m = 2(x+p0) - cw, c = m / 2b
            const int m = 2 * (x + al.p0) - al.cw;
            c = m / (2 * al.b);
        }
        lbase[e] = (c - cA) * NO;
        wl[e] = val[e] ? cell_weight(al, c, x) : 0.f;
    }
    const Tin *in = (const Tin *)d.in;
    const float nbf = (float)nb;
    const int nbm1 = nb - 1;
    const int64_t so = mc_div(rpi, rs.in_len);
    const int sr = (int)(rpi - so * rs.in_len);
    // descriptor fields of the row loop, held in scalar registers
    const McAxis aw = mc_uniform_axis(d.ax[D >= 2 ? D - 2 : 0]);
    void *const outp = mc_uniform_ptr(d.out);
    const int out_dt = mc_uniform(d.out_dt);
    const bool ntst = mc_uniform(d.ntst) != 0;
    const bool vecst = (out_dt == MC_F32) && (V % 4 == 0) && allv;
    // the unit's row chunks, one after another on the same staged LUTs; the
    // outer-row table is rebuilt for each chunk
    // (under per-kernel ranges the unit's 2^D corner ranges stay in
    // registers across its chunks too: each staging of 2^D LUTs, 32 KB at the
    // 4D workload, then serves a whole cell instead of a fifth of one)
    const int chA = chunk * d.mK, chB = mc_min(chA + d.mK, d.mCr);
    for (int ch = chA; ch < chB; ++ch) {
        const int64_t r0 = mc_div(rs.rows * ch, d.mCr), r1 = mc_div(rs.rows * (ch + 1), d.mCr);
        const int64_t o0 = mc_div(r0, rs.in_len);
        const int ocnt = r1 > r0 ? (int)(mc_div(r1 - 1, rs.in_len) - o0 + 1) : 0;
        if (ch > chA) __syncthreads();   // every reader of the previous table is done
        for (int j = threadIdx.x; j < ocnt; j += NT) {
            int32_t x[MC_MAXD];
            decode_outer(d, rs, o0 + j, x);
            int64_t off = 0;
            float cf[NOH];
            cf[0] = 1.0f;
            int n = 1;
#pragma unroll
            for (int i = 0; i < D - 2; ++i) {
                off += (int64_t)x[i] * ost[i];
                const float w = cell_weight(oax[i], cidx[i], x[i]);
                const float omw = 1.0f - w;
                // tensor product, axis i becomes the next lower-order bit
#pragma unroll
                for (int q = NOH - 1; q >= 0; --q) {
                    if (q < 2 * n) {
                        const float base = cf[q >> 1];
                        cf[q] = (q & 1) ? base * w : base * omw;
                    }
                }
                n *= 2;
            }
            otab[j].off = off;
#pragma unroll
            for (int q = 0; q < NOH; ++q) otab[j].coef[q] = cf[q];
        }
        __syncthreads();
        if (!tact) continue;
        const int64_t rstart = r0 + trow;
        int64_t o = mc_div(rstart, rs.in_len);
        int r = (int)(rstart - o * rs.in_len);
        // rows whose loads are in flight together (with NT threads and two
        // units per CU this keeps ~64 KiB of loads in flight per CU)
        constexpr int U = V >= 8 ? 2 : 4;
        for (int64_t row = rstart; row < r1; row += (int64_t)U * rpi) {
            int64_t offs[U];
            float win[U];
            float cfu[U][NOH];
            bool ok[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                ok[u] = row + (int64_t)u * rpi < r1;
                const OT &te = otab[ok[u] ? (int)(o - o0) : 0];
                const int xin = rs.in_lo + r;
                offs[u] = te.off + (int64_t)xin * rs.in_stride + xoff;
                win[u] = D >= 2 ? cell_weight(aw, cidx[D >= 2 ? D - 2 : 0], xin) : 0.f;
#pragma unroll
                for (int q = 0; q < NOH; ++q) cfu[u][q] = D >= 3 ? te.coef[q] : 1.0f;
                r += sr;
                o += so;
                if (r >= rs.in_len) {
                    r -= rs.in_len;
                    o += 1;
                }
            }
            float fu[U][V];
#pragma unroll
            for (int u = 0; u < U; ++u)
                if (ok[u]) load_chunk<Tin, V>(in + offs[u], fu[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                if (!ok[u]) break;
                float rc[NO];
                if constexpr (D == 1) {
                    rc[0] = 1.0f;
                } else {
                    const float w = win[u];
                    const float omw = 1.0f - w;
#pragma unroll
                    for (int q = 0; q < NOH; ++q) {
                        rc[2 * q] = cfu[u][q] * omw;
                        rc[2 * q + 1] = cfu[u][q] * w;
                    }
                }
                float y[V];
#pragma unroll
                for (int e = 0; e < V; ++e) {
                    const float fe = fu[u][e];
                    float Lv[NC];
                    if constexpr (AHR) {
#pragma unroll
                        for (int c = 0; c < NC; ++c)
                            Lv[c] = lut[__umul24(c, nb) + bin_of(fe, clo[c], csc[c], nbf, nbm1)];
                    } else {
                        const int b = bin_of(fe, glo, gsc, nbf, nbm1);
                        const float *p = lut + __umul24(b, SB) + lbase[e];
                        if constexpr (NO % 4 == 0) {
#pragma unroll
                            for (int c = 0; c < NC; c += 4) {
                                const float4 q = *reinterpret_cast<const float4 *>(p + c);
                                Lv[c] = q.x;
                                Lv[c + 1] = q.y;
                                Lv[c + 2] = q.z;
                                Lv[c + 3] = q.w;
                            }
                        } else if constexpr (NO % 2 == 0) {
#pragma unroll
                            for (int c = 0; c < NC; c += 2) {
                                const float2 q = *reinterpret_cast<const float2 *>(p + c);
                                Lv[c] = q.x;
                                Lv[c + 1] = q.y;
                            }
                        } else {
#pragma unroll
                            for (int c = 0; c < NC; ++c) Lv[c] = p[c];
                        }
                    }
                    float A = rc[0] * Lv[0], B = rc[0] * Lv[NO];
#pragma unroll
                    for (int c = 1; c < NO; ++c) {
                        A = __fmaf_rn(rc[c], Lv[c], A);
                        B = __fmaf_rn(rc[c], Lv[NO + c], B);
                    }
                    y[e] = __fmaf_rn(wl[e], B - A, A);
                }
                const int64_t off = offs[u];
                if (vecst) {
                    // streaming stores when the unit writes whole cache lines;
                    // otherwise write-back stores let L2 merge the parts of a
                    // line that neighbouring units write
                    if constexpr (V % 4 == 0) {
                        f4 *op = (f4 *)((float *)outp + off);
                        if (ntst) {
#pragma unroll
                            for (int q = 0; q < V / 4; ++q) {
                                f4 t = {y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]};
                                __builtin_nontemporal_store(t, op + q);
                            }
                        } else {
#pragma unroll
                            for (int q = 0; q < V / 4; ++q) op[q] = f4{y[4 * q], y[4 * q + 1], y[4 * q + 2], y[4 * q + 3]};
                        }
                    }
                } else {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (val[e]) store_elem(outp, out_dt, off + e, y[e]);
                }
                if constexpr (MET) {
#pragma unroll
                    for (int e = 0; e < V; ++e)
                        if (val[e]) macc.add(fu[u][e], out_value(out_dt, y[e]));
                }
            }
        }
    }
    if constexpr (MET) {
        __syncthreads();   // every reader of the staged tables is done
        met_flush<NT>(macc, smem, d.met + wu);
    }
}

template <typename Tin, int D, bool AHR, bool MET = false, int NT = mc_map_threads(AHR)>
__device__ void map_unit(const McVol &d, uint32_t wu, char *smem)
{
    constexpr int VM = mc_vec_elems((int)sizeof(Tin));
    if (d.vec == VM) map_unit_v<Tin, D, AHR, VM, MET, NT>(d, wu, smem);
    else map_unit_v<Tin, D, AHR, 1, MET, NT>(d, wu, smem);
}

// Generic interpolation (any D up to 8, or LUTs too large for LDS): one cell
// per unit, LUTs read from global memory, corners summed in index order.
template <typename Tin, bool AHR, bool MET = false>
__device__ void map_unit_generic(const McVol &d, uint32_t wu, char *smem)
{
    const int D = d.D, nb = d.nb;
    const int NC = 1 << D;
    int chunk, grp;
    int32_t cidx[MC_MAXD];
    RowSpace rs;
    map_unit_decode(d, wu, chunk, grp, cidx, rs);
    const McAxis &al = d.ax[D - 1];
    const int cl = grp;   // one cell per unit on the last axis (mG == 1)
    int xs, xe;
    mc_cell_range(al, cl, xs, xe);
    int64_t kst[MC_MAXD];
    int64_t kbase = 0;
    {
        int64_t s = 1;
#pragma unroll
        for (int i = MC_MAXD - 1; i >= 0; --i) {
            if (i <= D - 1) {
                kst[i] = s;
                s *= d.ax[i].n;
            } else {
                kst[i] = 0;
            }
        }
    }
#pragma unroll
    for (int i = 0; i < MC_MAXD; ++i) {
        if (i <= D - 2) kbase += (int64_t)cidx[i] * kst[i];
        if (i == D - 1) kbase += (int64_t)cl * kst[i];
    }
    float glo = 0.f, gsc = 0.f;
    if (!AHR) {
        glo = d.range[0];
        gsc = d.scale[0];
    }
    const int64_t r0 = mc_div(rs.rows * chunk, d.mCr), r1 = mc_div(rs.rows * (chunk + 1), d.mCr);
    const int xl = xe - xs;
    const int64_t nel = (r1 - r0) * xl;
    const float nbf = (float)nb;
    const int nbm1 = nb - 1;
    MetAcc macc;
    if constexpr (MET) macc.init();
    for (int64_t e = threadIdx.x; e < nel; e += MC_T) {
        const int64_t row = r0 + mc_div(e, xl);
        const int x = xs + (int)(e - (row - r0) * xl);
        // decode the row into outer coordinates
        int32_t xc[MC_MAXD];
        int64_t rr = row;
        int64_t off = x;
#pragma unroll
        for (int i = MC_MAXD - 2; i >= 0; --i) {
            if (i <= D - 2) {
                const int64_t q = mc_div(rr, rs.len[i]);
                xc[i] = rs.lo[i] + (int)(rr - q * rs.len[i]);
                rr = q;
                off += (int64_t)xc[i] * d.stride[i];
            }
        }
        float w[MC_MAXD];
#pragma unroll
        for (int i = 0; i < MC_MAXD; ++i) {
            if (i <= D - 2) w[i] = cell_weight(d.ax[i], cidx[i], xc[i]);
            if (i == D - 1) w[i] = cell_weight(al, cl, x);
        }
        const float v = load_elem(d.in, d.in_dt, off);
        float y = 0.0f;
        for (int c = 0; c < NC; ++c) {
            float coef = 1.0f;
            int64_t kid = kbase;
#pragma unroll
            for (int i = 0; i < MC_MAXD; ++i) {
                if (i <= D - 1) {
                    const int bit = (c >> (D - 1 - i)) & 1;
                    coef *= bit ? w[i] : 1.0f - w[i];
                    kid += bit ? kst[i] : 0;
                }
            }
            const float lo = AHR ? d.range[2 * kid] : glo;
            const float sc = AHR ? d.scale[kid] : gsc;
            y = __fmaf_rn(coef, d.lut[kid * nb + bin_of(v, lo, sc, nbf, nbm1)], y);
        }
        store_elem(d.out, d.out_dt, off, y);
        if constexpr (MET) macc.add(v, out_value(d.out_dt, y));
    }
    if constexpr (MET) met_flush<MC_T>(macc, smem, d.met + wu);
}

}  // namespace mc
