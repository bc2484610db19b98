// Volume descriptor and geometry helpers shared by the host runtime and the
// gfx950 kernels of the MCLAHE library.  Plain-old-data only: the same struct
// is passed by value to the per-pass kernels and stored in a device table for
// the batched kernels.
#pragma once
#include <stdint.h>

#if defined(__HIPCC__)
#include <hip/hip_runtime.h>
#define MC_HD __host__ __device__ __forceinline__
#else
#define MC_HD inline
#endif

// Device code addresses the volume's buffers in the global address space
// (the host sees plain pointers; the layout is the same).
#if defined(__HIP_DEVICE_COMPILE__)
#define MC_GLOBAL __attribute__((address_space(1)))
#else
#define MC_GLOBAL
#endif

#define MC_MAXD 8          // dimensions supported

// A device buffer pointer as the descriptor holds it.
template <typename T>
MC_HD MC_GLOBAL T *mc_gp(T *p) { return (MC_GLOBAL T *)p; }
#define MC_T 256           // threads per work-group (4 wavefronts of 64)
#define MC_MAP_T 512       // threads per work-group of the LDS-staged map with
                           // a global range (its LDS bounds the units per CU:
                           // bigger groups keep more waves in flight); the
                           // adaptive-range map, heavier in registers, uses MC_T
#define MC_OMAX 256        // outer-row table entries per work unit
#define MC_STAGE 8         // loads a thread keeps in flight while staging
                           // per-kernel arrays (LUTs, partials) of a unit
#define MC_LDS_BUDGET (64 * 1024)   // LDS a work unit may use (bytes)
#define MC_NUM_CU 256      // MI355X compute units (tiling target)

enum { MC_U8 = 0, MC_U16 = 1, MC_F32 = 2 };
enum { MC_GHR = 0, MC_AHR = 1 };
enum { MC_REDIST_EQUAL = 0, MC_REDIST_REPEATED = 1, MC_REDIST_INTEGER = 2 };

// One axis of the padded kernel grid: size s, kernel b, padding p0 before and
// p1 after (Eq. 1-2), n = (s + p0 + p1) / b kernels; cw = twice the offset of
// a kernel's centre from its first sample: b - 1 (centre in the middle), or
// 2 * (b / 2) for the comparison variant with the centre at b / 2.
struct McAxis {
    int32_t s, b, p0, p1, n, cw;
};

// Original-coordinate footprint of kernel k along one axis: every padded
// position of the kernel mirrors to an x in [lo, hi); x in [olo, ohi) is hit
// twice (once directly, once through the mirror), every other x once.
struct McBox {
    int32_t lo, hi, olo, ohi;
};

MC_HD int32_t mc_min(int32_t a, int32_t b) { return a < b ? a : b; }
MC_HD int32_t mc_max(int32_t a, int32_t b) { return a > b ? a : b; }

MC_HD McBox mc_kernel_box(const McAxis &a, int32_t k)
{
    const int32_t q0 = k * a.b, q1 = q0 + a.b;
    // direct part: q in [max(q0,p0), min(q1,p0+s)) -> x = q - p0
    const int32_t d0 = mc_max(q0, a.p0) - a.p0, d1 = mc_min(q1, a.p0 + a.s) - a.p0;
    // mirrored part (a window of b <= s voxels holds at most one fold)
    int32_t m0 = 0, m1 = 0;
    if (q0 < a.p0) {                       // start fold: x = p0 - 1 - q
        m0 = a.p0 - mc_min(q1, a.p0);
        m1 = a.p0 - q0;
    } else if (q1 > a.p0 + a.s) {          // end fold: x = 2s - 1 - (q - p0)
        m0 = 2 * a.s + a.p0 - q1;
        m1 = 2 * a.s + a.p0 - mc_max(q0, a.p0 + a.s);
    }
    McBox r;
    const bool hd = d0 < d1, hm = m0 < m1;
    r.lo = hd ? (hm ? mc_min(d0, m0) : d0) : m0;
    r.hi = hd ? (hm ? mc_max(d1, m1) : d1) : m1;
    r.olo = mc_max(d0, m0);
    r.ohi = mc_min(d1, m1);
    if (!(hd && hm) || r.olo >= r.ohi) r.olo = r.ohi = r.lo;
    return r;
}

// Multiplicity (0, 1 or 2) of original coordinate x in kernel k's footprint.
MC_HD int32_t mc_mult(const McBox &bx, int32_t x)
{
    return (x >= bx.lo && x < bx.hi) ? 1 + (x >= bx.olo && x < bx.ohi) : 0;
}

// Interpolation cell c (voxels whose lower neighbour kernel is c) along one
// axis: x in [lo, hi).  Kernel centres sit at k*b + (b-1)/2 in padded
// coordinates, so the cell starts at b*c + floor(b/2) - p0.
MC_HD void mc_cell_range(const McAxis &a, int32_t c, int32_t &lo, int32_t &hi)
{
    lo = a.b * c + a.b / 2 - a.p0;
    hi = lo + a.b;
    if (lo < 0) lo = 0;
    if (hi > a.s) hi = a.s;
}

// Doubled offset of x from the lower kernel centre of its cell c:
// m = 2(x + p0) - cw - 2bc, in [0, 2b); weight = m / (2b).  (Both centre
// conventions give the same cells: the first voxel at or past a centre.)
MC_HD int32_t mc_cell_m(const McAxis &a, int32_t c, int32_t x)
{
    return 2 * (x + a.p0) - a.cw - 2 * a.b * c;
}

// LDS stride (floats) of one bin's row in the staged GHR LUTs: nlk last-axis
// kernels x NO outer corners, padded to an odd number of read units (16-byte
// reads when NO >= 4) so that lanes reading different bins hit different
// bank groups.
MC_HD int32_t mc_lut_stride(int32_t nlk, int32_t NO)
{
    const int32_t cw = NO >= 4 ? 4 : NO;
    int32_t q = nlk * NO / cw;
    if ((q & 1) == 0) q += 1;
    return q * cw;
}

// LDS words of one slot (kernel) of a histogram unit: n bins x R replicas,
// plus one word so that the stride is odd and slots spread over the banks.
MC_HD int32_t mc_hist_slot_stride(int32_t nb, int32_t R) { return nb * R + 1; }

// Elements per chunk of a row: 16 bytes (4 floats, 8 uint16), but 8 uint8,
// which keeps the per-element registers of a thread bounded.
MC_HD constexpr int mc_vec_elems(int esize) { return esize == 1 ? 8 : 16 / esize; }

// Work-group size of the LDS-staged map kernels.
MC_HD constexpr int mc_map_threads(bool ahr) { return ahr ? MC_T : MC_MAP_T; }

// Partial statistics of one work unit for the contrast metrics: minimum,
// maximum and float64 sum of the input ([0]) and of the stored output ([1])
// over the unit's voxels (the same record the metrics' own range pass
// writes per work-group).
struct McMetPart {
    float mn[2], mx[2];
    double sum[2];
};

// Everything the kernels need about one volume.
struct McVol {
    // ---- problem -----------------------------------------------------------
    int32_t D, nb, in_dt, out_dt, mode, has_user_range;
    float user_lo, user_hi;
    int64_t clipC;            // clip count C = floor(clip * K)
    int64_t K;                // voxels per kernel
    int32_t redist, rounds;   // redistribution of the excess (MC_REDIST_*), and
                              // the most rounds of the repeated variant
    McAxis ax[MC_MAXD];
    int64_t stride[MC_MAXD];  // element strides (C-contiguous)
    int64_t nvox, nker;
    int32_t vec;              // elements per vector chunk (1 or mc_vec_elems)
    int32_t path;             // 0 = LDS-staged fast map, 1 = generic map
    // ---- histogram / adaptive-range work units ------------------------------
    int32_t hG, hP, hS, hCr;  // kernels per segment, parts per kernel,
                              // segments on the last axis, row chunks
    int32_t hR, hPeel;        // LDS replicas, aggregation rounds
    int32_t wk0, wc0;         // window on axis 0 (chunked runs): first kernel
                              // layer of the histogram units, first cell layer
                              // of the interpolation units (0 for whole volumes)
    int32_t ntst;             // 1: output row segments are whole 64-byte blocks
                              //    -> streaming (non-temporal) stores
    int32_t vhist;            // 1: uint8 input counted per value (256 slots per
                              //    kernel, no range pass); the clip pass takes
                              //    the range and re-bins the values
    int64_t hCols;            // kernel columns (prod of n_i, i < D-1)
    uint32_t n_hist_wu;       // hCols * hS * hCr
    uint32_t n_range_wu;      // GHR min/max blocks (0 if a user range is given)
    // ---- interpolation work units -------------------------------------------
    int32_t mG, mS, mCr, mP;  // cells per group, segments on the last axis,
                              // row chunks, parts per cell (mP > 1: mG = 1)
    int32_t mK, mU;           // row chunks per unit (on one LUT staging),
                              // units per (cell column, segment) = ceil(mCr/mK)
    int64_t mCols;            // cell columns (prod of n_i - 1, i < D-1)
    uint32_t n_map_wu;        // mCols * mS * mU
    uint32_t n_clip_wu;       // = nker
    // ---- buffers (device memory; kernels address them as global memory,
    //      whichever memory the descriptor itself is read from) ------------
    const MC_GLOBAL void *in;
    MC_GLOBAL void *out;
    MC_GLOBAL uint32_t *part;           // [n_hist_wu][hG][nb]   partial histograms
    MC_GLOBAL float *rpart;             // GHR: [n_range_wu][2]; AHR: [n_hist_wu][hG][2]
    MC_GLOBAL uint32_t *hist;           // [nker][nb]
    MC_GLOBAL unsigned long long *clipped;  // [nker][nb]
    MC_GLOBAL float *lut;               // [nker][nb]
    MC_GLOBAL float *range;             // GHR: [2]; AHR: [nker][2]
    MC_GLOBAL float *scale;             // GHR: [1]; AHR: [nker]
    MC_GLOBAL McMetPart *met;           // contrast metrics: [n_map_wu] partials of the
                                        // interpolation units (NULL: not computed)
};


// Batched descriptor table (device memory, uploaded per call): a header, one
// record per batched launch, the launches' index arrays, then the volume
// descriptors.  A batched launch runs one pass for every volume of one kernel
// class (the template instance the per-volume path would launch).
#define MC_PHASES 4
struct McBatchHdr {
    uint32_t nvol, nlaunch;
    uint32_t o_persist;   // byte offset of the persistent launch's table (McPersistHdr)
    uint32_t pad_;
};
struct McLaunchRec {
    uint32_t phase;    // 0 range, 1 histogram, 2 clip/CDF, 3 map
    uint32_t n;        // volumes in this launch
    uint32_t list;     // offset (in uint32) of the volume index list [n]
    uint32_t pre;      // offset (in uint32) of the unit prefix sums [n + 1]
    uint32_t units;    // work-groups of the launch (= pre[n])
    uint32_t pad_[3];
};

// What a batched kernel receives (by value).
struct McBatchSrc {
    const McVol *vols;
    const uint32_t *list;
    const uint32_t *pre;
    uint32_t n, pad_;
};

// Units of pass ph of a volume: 0 range, 1 histogram, 2 clip/CDF, 3 map.
MC_HD uint32_t mc_phase_units(const McVol &v, int ph)
{
    return ph == 0 ? (v.vhist ? 0u : v.mode == MC_AHR ? v.n_hist_wu : v.n_range_wu)
         : ph == 1 ? v.n_hist_wu : ph == 2 ? v.n_clip_wu : v.n_map_wu;
}

// Entry j owning unit r of a launch: the largest j with pre[j] <= r, where
// pre holds the prefix sums of the units (pre[0] = 0, pre[n] = all units).
MC_HD uint32_t mc_batch_volume(const uint32_t *pre, uint32_t n, uint32_t r)
{
    uint32_t lo = 0, hi = n;
    while (hi - lo > 1) {
        const uint32_t mid = (lo + hi) / 2;
        if (pre[mid] <= r) lo = mid;
        else hi = mid;
    }
    return lo;
}
