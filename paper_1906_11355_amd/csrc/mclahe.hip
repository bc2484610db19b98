// Host runtime and C ABI of the MI355X MCLAHE library (see include/mclahe.h).
//
// mclahe_run        : four stream-ordered launches (range, histogram,
//                     clip/CDF/LUT, interpolation), one work-group per unit.
// mclahe_run_batched: the same four passes for a whole batch of volumes,
//                     one launch per pass covering the units of every volume,
//                     replayed from a cached hipGraph after one copy of the
//                     batch's descriptor table.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <set>
#include <new>
#include <string>
#include <vector>

#include "../../include/mclahe.h"
#include "mc_desc.h"
#include "mc_kernels.h"
#include "mc_persist.h"

// ------------------------------------------------------------------ errors --
static thread_local std::string g_err;

static mclahe_status fail(mclahe_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

mclahe_status mc_fail(mclahe_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return s;
}

void mc_clear_error() { g_err.clear(); }

#define HIPCHK(call)                                                                     \
    do {                                                                                 \
        hipError_t e_ = (call);                                                          \
        if (e_ != hipSuccess)                                                            \
            return fail(MCLAHE_ERROR_HIP, "%s failed: %s", #call, hipGetErrorString(e_)); \
    } while (0)

// ------------------------------------------------------------------- plan --
struct mclahe_plan_s {
    int D;
    int64_t shape[MC_MAXD], ks[MC_MAXD];
    int nb;
    double clip;
    int mode;
    int has_ur;
    float ur[2];
    int in_dt, out_dt;
    McAxis ax[MC_MAXD];
    int64_t stride[MC_MAXD];
    int64_t nvox, nker, K, clipC, ncells;
    mclahe_tuning tune;   // requested for per-volume runs (0 = default)
    mclahe_tuning btune;  // requested for batched runs (0 = default)
    int redist = MC_REDIST_EQUAL, rounds = 1, centre_half = 0;   // method variant
    // Derived work decompositions (descriptors without pointers).  Vector
    // loads need 16-byte aligned buffers and bound how long a unit's row
    // segment may be (MC_T chunks of V elements); buffers at any other
    // address take the scalar decomposition, whose segments fit MC_T single
    // elements.  Batched launches default to coarser units (many volumes
    // fill the chip together).
    McVol v, v1;     // per-volume runs: vector loads, scalar loads
    McVol bv, bv1;   // batched runs: vector loads, scalar loads
    // one workspace layout serves all four decompositions
    uint64_t o_part, o_rpart, o_hist, o_clipped, o_lut, o_range, o_scale, total;
};

// Clip count C = floor(clip * K) (Algorithm 1's clip limit as a fraction of
// the kernel's voxel count).  A clip limit is written as a decimal whose
// binary value may fall a rounding error short of it (0.02 * 270000 must
// give 5400, 0.29 * 100 must give 29), so a product within a relative 2^-40
// below an integer counts as that integer; C is capped at K (at K or above
// no bin is clipped).
static int64_t clip_count(double clip, int64_t K)
{
    const double c = clip * (double)K;
    if (!(c < (double)K)) return K;   // no bin can exceed K: nothing is clipped
    int64_t C = (int64_t)c;
    if ((double)(C + 1) - c <= std::ldexp(c, -40)) ++C;
    return C;
}

// Default minimum voxels per histogram / interpolation work unit: a unit's
// fixed cost (staging and flushing its LDS arrays) dominates smaller ones.
// Batched launches fill the chip with the units of many volumes, so they take
// coarser units.
static const int64_t kUnitVoxPlain = 16384, kUnitVoxBatch = 65536;
// Voxels per interpolation unit a batched volume aims at under a global range
// (a unit then stages its LUTs for about as many rows as at the 4D headline)
static const int64_t kMapUnitVoxBatch = 65536;
// Polls of one wait of the persistent launch before the run gives up (each
// poll an atomic and a short sleep: on the order of a second in all)
static const uint32_t kPersistSpins = 1u << 20;
// unit columns the plain interpolation pass keeps at least (one per CU)
static const int64_t kMinMapCols = 256;

static size_t esize(int dt) { return dt == MC_U8 ? 1 : dt == MC_U16 ? 2 : 4; }
static uint64_t align256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

// Header bytes of a histogram unit's LDS (see mc::hist_lds).
static size_t hist_lds_header() { return sizeof(mc::HistOTab) * MC_OMAX + 4 * 2 * MC_T + 4 * 64 * 2 + 4 * 128; }

static size_t map_otab_bytes(int D)
{
    switch (D) {
    case 1: return sizeof(mc::MapOTab<1>) * MC_OMAX;
    case 2: return sizeof(mc::MapOTab<2>) * MC_OMAX;
    case 3: return sizeof(mc::MapOTab<3>) * MC_OMAX;
    default: return sizeof(mc::MapOTab<4>) * MC_OMAX;
    }
}

static size_t map_lut_bytes(const mclahe_plan_s *p, int mG)
{
    const int D = p->D;
    if (p->mode == MC_AHR) return (size_t)(1 << D) * p->nb * 4;
    return (size_t)p->nb * mc_lut_stride(mG + 1, 1 << (D - 1)) * 4;
}

// Extent of the last-axis hist segment made of kernels [kA,kB).
static void seg_extent(const McAxis &a, int kA, int kB, int &xs, int &xe)
{
    xs = INT32_MAX;
    xe = -1;
    for (int k = kA; k < kB; ++k) {
        McBox b = mc_kernel_box(a, k);
        xs = std::min(xs, b.lo);
        xe = std::max(xe, b.hi);
    }
}

// Chunks of V elements a segment [xs, xe) spans.
static int seg_chunks(int xs, int xe, int V) { return (xe + V - 1) / V - xs / V; }

// Derive a work decomposition from tuning t, with default work units of at
// least unit_vox voxels, for vector loads (vector: chunks of mc_vec_elems
// elements when the last axis holds at least one) or scalar loads.  Under
// a global range, interpolation units run row chunks on one staging of
// their LUTs: by default as many as leave map_units units for the volume.
static mclahe_status derive_core(const mclahe_plan_s *p, const mclahe_tuning &t, int64_t unit_vox,
                                 int64_t min_map_cols, int64_t map_units, bool vector, bool spread, McVol &v)
{
    memset(&v, 0, sizeof v);
    const int D = p->D;
    v.D = D;
    v.nb = p->nb;
    v.in_dt = p->in_dt;
    v.out_dt = p->out_dt;
    v.mode = p->mode;
    v.has_user_range = p->has_ur;
    v.user_lo = p->ur[0];
    v.user_hi = p->ur[1];
    v.clipC = p->clipC;
    v.K = p->K;
    v.redist = p->redist;
    v.rounds = p->rounds;
    for (int i = 0; i < MC_MAXD; ++i) {
        v.ax[i] = p->ax[i];
        v.stride[i] = p->stride[i];
    }
    v.nvox = p->nvox;
    v.nker = p->nker;
    const McAxis &al = p->ax[D - 1];
    const int vmax = mc_vec_elems((int)esize(p->in_dt));
    // chunks start at any element of a row (global memory takes unaligned
    // wide loads); the chunk that would run past a row's end is read as the
    // row's last vmax elements, so a row needs at least one whole chunk
    const int V = (vector && al.s >= vmax) ? vmax : 1;
    v.vec = V;
    const int maxchunks = MC_T - 1;

    // ---- histogram units --------------------------------------------------
    // LDS replicas of the histograms (lane l updates replica l mod R): two
    // halve the same-address conflicts of lanes that bin equal values
    // (headline histogram pass 0.230 -> 0.220 ms, the 4D class of the batched
    // mix 1.100 -> 1.058 ms); more did not pay for zeroing and summing them
    int R = t.hist_copies > 0 ? t.hist_copies : 2;
    if (R != 1 && R != 2 && R != 4 && R != 8) return fail(MCLAHE_ERROR_INVALID_VALUE, "hist_copies must be 1, 2, 4 or 8");
    // uint8 input is counted per value (256 slots per kernel) and re-binned
    // by the clip pass, which also takes the range: no range pass.  The slot
    // sizes below fit both that and a bin histogram (the out-of-core run
    // counts bins with the same units).
    v.vhist = p->in_dt == MC_U8 ? 1 : 0;
    const int nbs = v.vhist ? std::max(p->nb, 256) : p->nb;
    const size_t hdr = hist_lds_header();
    while (R > 1 && hdr + (size_t)mc_hist_slot_stride(nbs, R) * 4 > MC_LDS_BUDGET) R /= 2;
    if (hdr + (size_t)mc_hist_slot_stride(nbs, 1) * 4 > MC_LDS_BUDGET)
        return fail(MCLAHE_ERROR_NOT_SUPPORTED, "n_bins=%d needs more LDS than a work-group may use", p->nb);
    int Gmax = (int)std::min<size_t>(64, (MC_LDS_BUDGET - hdr) / ((size_t)mc_hist_slot_stride(nbs, R) * 4));
    Gmax = std::max(1, std::min(Gmax, al.n));
    int G = 0;
    for (int g = Gmax; g >= 1; --g) {
        bool ok = true;
        for (int kA = 0; kA < al.n && ok; kA += g) {
            int xs, xe;
            seg_extent(al, kA, std::min(kA + g, al.n), xs, xe);
            ok = seg_chunks(xs, xe, V) <= maxchunks;
        }
        if (ok) {
            G = g;
            break;
        }
    }
    int P = 1;
    if (G == 0) {   // one kernel is too long for a work-group row: split it
        G = 1;
        int maxlen = 0;
        for (int k = 0; k < al.n; ++k) {
            McBox b = mc_kernel_box(al, k);
            maxlen = std::max(maxlen, b.hi - b.lo);
        }
        P = 2;
        for (;; ++P) {
            bool ok = true;
            for (int k = 0; k < al.n && ok; ++k) {
                McBox b = mc_kernel_box(al, k);
                const int len = b.hi - b.lo;
                for (int pp = 0; pp < P && ok; ++pp) {
                    const int xs = b.lo + (int)((int64_t)len * pp / P);
                    const int xe = b.lo + (int)((int64_t)len * (pp + 1) / P);
                    ok = seg_chunks(xs, xe, V) <= maxchunks;
                }
            }
            if (ok) break;
        }
    }
    v.hP = P;
    v.hR = R;
    // hist_peel: 0 = default (no aggregation), k >= 1 = k - 1 rounds
    v.hPeel = t.hist_peel > 1 ? 1 : 0;   // one aggregation round (a second only spilled)
    v.hCols = 1;
    int64_t omax_h = 1, rmax_h = 1;
    for (int i = 0; i < D - 1; ++i) {
        v.hCols *= p->ax[i].n;
        int mx = 0;
        for (int k = 0; k < p->ax[i].n; ++k) {
            McBox b = mc_kernel_box(p->ax[i], k);
            mx = std::max(mx, b.hi - b.lo);
        }
        rmax_h *= mx;
        if (i <= D - 3) omax_h *= mx;
    }
    const int64_t crmin_h = std::max<int64_t>(1, (omax_h + MC_OMAX - 5) / (MC_OMAX - 4));
    // default row split: ~2048 units, but no unit under ~16K voxels (the
    // fixed cost of a unit, zeroing and flushing its LDS histograms, then
    // dominates; measured on the 2D 512x512 and 3D 256x256x128 workloads)
    auto split_for = [&](int g, bool tuned, int64_t &segs, int64_t &cr) {
        segs = P == 1 ? (al.n + g - 1) / g : (int64_t)al.n * P;
        int64_t seglen = 0;
        for (int j = 0; j < segs; ++j) {
            int xs, xe;
            if (P == 1) {
                seg_extent(al, j * g, std::min(j * g + g, al.n), xs, xe);
                seglen = std::max<int64_t>(seglen, (int64_t)(xe - xs));
            } else {
                const McBox bx = mc_kernel_box(al, j / P);
                seglen = std::max<int64_t>(seglen, ((int64_t)(bx.hi - bx.lo) + P - 1) / P);
            }
        }
        const int64_t cr_units = (2048 + v.hCols * segs - 1) / (v.hCols * segs);
        const int64_t cr_work = std::max<int64_t>(1, rmax_h * seglen / unit_vox);
        cr = tuned && t.hist_rows_split > 0 ? t.hist_rows_split : std::min(cr_units, cr_work);
        cr = std::max<int64_t>(cr, crmin_h);
        cr = std::min<int64_t>(cr, std::max<int64_t>(rmax_h, crmin_h));
    };
    // A volume alone takes fewer kernels per segment when the widest segments
    // leave fewer units than compute units: a unit then zeroes and flushes
    // fewer histograms and its work-group has fewer rows to walk, and the
    // units spread over the chip (2D 512x512 uint8, 9 kernels per row:
    // segments of 9 kernels in 18 units, 20.6 us, against single kernels in
    // 81 units, 15.6 us).  The largest segment that still gives a unit per
    // compute unit is kept, else the one giving the most units (counted with
    // the default row split, so that the choice does not depend on tuning).
    if (spread && P == 1) {
        int best = G;
        int64_t best_units = -1;
        for (int g = G; g >= 1; --g) {
            int64_t segs, cr;
            split_for(g, false, segs, cr);
            const int64_t u = v.hCols * segs * cr;
            if (u >= MC_NUM_CU) {
                best = g;
                break;
            }
            if (u > best_units) {
                best_units = u;
                best = g;
            }
        }
        G = best;
    }
    v.hG = G;
    int64_t segs = 0, cr = 0;
    split_for(G, true, segs, cr);
    v.hS = (int)segs;
    if (cr > (1 << 20)) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "row split too large");
    v.hCr = (int)cr;
    const int64_t nhu = v.hCols * v.hS * v.hCr;
    if (nhu >= (int64_t)1 << 31) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "too many histogram units");
    v.n_hist_wu = (uint32_t)nhu;
    if (p->mode == MC_GHR) {
        v.n_range_wu = p->has_ur || v.vhist ? 0 : (uint32_t)std::min<int64_t>(1024, std::max<int64_t>(1, p->nvox / (MC_T * 64)));
    } else {
        v.n_range_wu = 0;
    }
    v.n_clip_wu = (uint32_t)p->nker;

    // ---- interpolation units ----------------------------------------------
    const size_t otab = map_otab_bytes(D);
    const bool fast = D <= 4 && otab + map_lut_bytes(p, 1) <= MC_LDS_BUDGET;
    v.path = fast ? 0 : 1;
    const int ncl = al.n - 1;  // cells on the last axis
    int64_t ocols = 1;         // interpolation cells on the outer axes
    for (int i = 0; i < D - 1; ++i) ocols *= p->ax[i].n - 1;
    int mG = 1;
    if (fast && p->mode == MC_GHR) {
        // default: the largest group that fits, but small enough that the
        // volume has min_map_cols unit columns before any row split (a small
        // volume in few wide units leaves most of the chip idle: 2D 512x512
        // uint8, 8 cells per axis, groups of 8 -> 1: 40 -> 35 us per step)
        int want = t.map_group > 0 ? t.map_group : ncl;
        want = std::min(want, ncl);
        for (int g = want; g >= 1; --g) {
            if (otab + map_lut_bytes(p, g) > MC_LDS_BUDGET) continue;
            if (g > 1 && t.map_group <= 0 && ocols * ((ncl + g - 1) / g) < min_map_cols) continue;
            bool ok = true;
            for (int cA = 0; cA < ncl && ok; cA += g) {
                int xs, xe, tmp;
                mc_cell_range(al, cA, xs, tmp);
                mc_cell_range(al, std::min(cA + g, ncl) - 1, tmp, xe);
                ok = seg_chunks(xs, xe, V) <= maxchunks;
            }
            if (ok) {
                mG = g;
                break;
            }
        }
    }
    int mP = 1;
    if (fast) {   // a cell too long for one work-group row is split in parts
        for (;; ++mP) {
            bool ok = true;
            for (int c = 0; c < ncl && ok; ++c) {
                int lo, hi;
                mc_cell_range(al, c, lo, hi);
                for (int pp = 0; pp < mP && ok; ++pp) {
                    const int xs = lo + (int)((int64_t)(hi - lo) * pp / mP);
                    const int xe = lo + (int)((int64_t)(hi - lo) * (pp + 1) / mP);
                    ok = seg_chunks(xs, xe, V) <= maxchunks;
                }
            }
            if (ok) break;
        }
        if (mP > 1) mG = 1;
    }
    v.mG = mG;
    v.mP = mP;
    // streaming stores only when every unit writes whole rows of whole lines
    v.ntst = 0;
    if (fast && mP == 1) {   // streaming stores when every row segment is whole 64-byte blocks
        bool ok = ((int64_t)al.s * (int64_t)esize(p->out_dt)) % 64 == 0;
        for (int cA = 0; cA < ncl && ok; cA += mG) {
            int xs, xe, tmp;
            mc_cell_range(al, cA, xs, tmp);
            mc_cell_range(al, std::min(cA + mG, ncl) - 1, tmp, xe);
            ok = ((int64_t)xs * (int64_t)esize(p->out_dt)) % 64 == 0 && ((int64_t)xe * (int64_t)esize(p->out_dt)) % 64 == 0;
        }
        v.ntst = ok ? 1 : 0;
    }
    v.mS = mP > 1 ? ncl * mP : (ncl + mG - 1) / mG;
    v.mCols = 1;
    int64_t omax_m = 1, rmax_m = 1;
    for (int i = 0; i < D - 1; ++i) {
        v.mCols *= p->ax[i].n - 1;
        rmax_m *= p->ax[i].b;
        if (i <= D - 3) omax_m *= p->ax[i].b;
    }
    const int64_t crmin_m = fast ? std::max<int64_t>(1, (omax_m + MC_OMAX - 5) / (MC_OMAX - 4)) : 1;
    // default row split: enough chunks for ~2048 units, but no chunk under
    // ~16K voxels (a unit's LUT staging dominates small ones); under a global
    // range also chunks of at most ~800 rows, the fastest measured at the 4D
    // workload (a unit runs several chunks on one LUT staging)
    int64_t segw = 0;   // widest last-axis extent of a unit
    for (int cA = 0; cA < ncl; cA += mG) {
        int xs, xe, tmp;
        mc_cell_range(al, cA, xs, tmp);
        mc_cell_range(al, std::min(cA + mG, ncl) - 1, tmp, xe);
        segw = std::max<int64_t>(segw, xe - xs);
    }
    if (mP > 1) segw = (segw + mP - 1) / mP;
    int64_t mcr = std::min<int64_t>((2048 + v.mCols * v.mS - 1) / (v.mCols * v.mS),
                                    std::max<int64_t>(1, rmax_m * segw / unit_vox));
    if (fast && p->mode == MC_GHR) mcr = std::max<int64_t>(mcr, (rmax_m + 799) / 800);
    if (t.map_rows_split > 0) mcr = t.map_rows_split;
    mcr = std::max<int64_t>(mcr, crmin_m);
    mcr = std::min<int64_t>(mcr, std::max<int64_t>(rmax_m, crmin_m));
    v.mCr = (int)mcr;
    // row chunks per unit: each unit stages its LUTs once for mK chunks.
    // Default: as many as keep >= map_units units (1024 for one volume, four
    // per CU; fewer for a volume of a batch, whose units share the chip with
    // the others' and would otherwise stage their LUTs for few rows)
    int mk = 1;
    if (fast) {
        if (t.map_unit_chunks > 0) {
            mk = t.map_unit_chunks;
        } else {
            const int64_t want_u = std::max<int64_t>(1, (map_units + v.mCols * v.mS - 1) / (v.mCols * v.mS));
            mk = (int)((mcr + want_u - 1) / want_u);
        }
        mk = std::max(1, std::min(mk, v.mCr));
    }
    v.mK = mk;
    v.mU = (v.mCr + mk - 1) / mk;
    const int64_t nmu = v.mCols * v.mS * v.mU;
    if (nmu >= (int64_t)1 << 31) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "too many map units");
    v.n_map_wu = (uint32_t)nmu;

    return MCLAHE_SUCCESS;
}

// Words of the per-unit partial histograms and floats of the range partials
// a decomposition writes.
static uint64_t part_words(const McVol &v)
{
    return (uint64_t)v.n_hist_wu * v.hG * (uint64_t)(v.vhist ? std::max(v.nb, 256) : v.nb);
}
static uint64_t rpart_floats(const McVol &v)
{
    if (v.vhist) return (uint64_t)v.n_hist_wu * 2;   // GHR: one (min, max) per unit
    return v.mode == MC_GHR ? (uint64_t)std::max<uint32_t>(v.n_range_wu, 1) * 2 : (uint64_t)v.n_hist_wu * v.hG * 2;
}

// LDS bytes of pass ph (0 range, 1 histogram, 2 clip, 3 map) under v.
static size_t pass_lds(const mclahe_plan_s *p, const McVol &v, int ph)
{
    const size_t hist = hist_lds_header() + (size_t)v.hG * mc_hist_slot_stride(v.vhist ? 256 : v.nb, v.hR) * 4;
    switch (ph) {
    case 0: return p->mode == MC_AHR ? hist : 2 * MC_T * 4;
    case 1: return hist;
    case 2: return MC_T * 8 + (v.vhist ? (size_t)v.nb * 4 : 0);   // + the re-binned histogram
    default: return v.path == 0 ? map_otab_bytes(p->D) + map_lut_bytes(p, v.mG) : 0;
    }
}

// All four decompositions, then one workspace layout that fits each of them.
// The per-kernel arrays come first (their offsets depend only on the
// problem), the per-unit partials last, sized for the largest decomposition.
static mclahe_status derive(mclahe_plan_s *p)
{
    mclahe_status s;
    const int64_t bmu = std::max<int64_t>(1, p->nvox / kMapUnitVoxBatch);
    if ((s = derive_core(p, p->btune, kUnitVoxBatch, 1, bmu, true, false, p->bv))) return s;
    if ((s = derive_core(p, p->btune, kUnitVoxBatch, 1, bmu, false, false, p->bv1))) return s;
    if ((s = derive_core(p, p->tune, kUnitVoxPlain, kMinMapCols, 1024, true, true, p->v))) return s;
    if ((s = derive_core(p, p->tune, kUnitVoxPlain, kMinMapCols, 1024, false, true, p->v1))) return s;
    uint64_t pw = 0, rf = 0;
    for (const McVol *d : {&p->v, &p->v1, &p->bv, &p->bv1}) {
        pw = std::max(pw, part_words(*d));
        rf = std::max(rf, rpart_floats(*d));
    }
    uint64_t o = 0;
    p->o_hist = o;
    o = align256(o + (uint64_t)p->nker * p->nb * 4);
    p->o_clipped = o;
    o = align256(o + (uint64_t)p->nker * p->nb * 8);
    p->o_lut = o;
    o = align256(o + (uint64_t)p->nker * p->nb * 4);
    p->o_range = o;
    o = align256(o + (p->mode == MC_AHR ? (uint64_t)p->nker * 2 : 2) * 4);
    p->o_scale = o;
    o = align256(o + (p->mode == MC_AHR ? (uint64_t)p->nker : 1) * 4);
    p->o_part = o;
    o = align256(o + pw * 4);
    p->o_rpart = o;
    o = align256(o + rf * 4);
    p->total = o;
    return MCLAHE_SUCCESS;
}

// Wide loads and stores work at any element address (the HSA runtime runs
// the GPU in unaligned-access mode), so the vector decomposition serves any
// buffers; the scalar one remains for rows shorter than one chunk.
static bool vec_aligned(const mclahe_plan_s *p, const void *in, const void *out)
{
    (void)p;
    (void)in;
    (void)out;
    return true;
}

// A copy of the plan that carries the batched decompositions, for the
// batched entry points (same problem, same bits, coarser default units).
static void batch_view(const mclahe_plan_s *p, mclahe_plan_s &q)
{
    q = *p;
    q.v = p->bv;
    q.v1 = p->bv1;
}

// Pointers of a run's descriptor.
static void bind(const mclahe_plan_s *p, McVol &v, const void *in, void *out, char *ws)
{
    v = vec_aligned(p, in, out) ? p->v : p->v1;
    v.in = mc_gp(in);
    v.out = mc_gp(out);
    v.part = mc_gp((uint32_t *)(ws + p->o_part));
    v.rpart = mc_gp((float *)(ws + p->o_rpart));
    v.hist = mc_gp((uint32_t *)(ws + p->o_hist));
    v.clipped = mc_gp((unsigned long long *)(ws + p->o_clipped));
    v.lut = mc_gp((float *)(ws + p->o_lut));
    v.range = mc_gp((float *)(ws + p->o_range));
    v.scale = mc_gp((float *)(ws + p->o_scale));
}

// Kernel selection lives in the per-dtype translation units (k_plain_*.hip).
#include "mc_launch.h"
#include "mc_plain_kernels.h"

__global__ __launch_bounds__(MC_T) void k_clip(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::clip_unit(d, blockIdx.x, smem);
}
__global__ __launch_bounds__(MC_T) void k_clip_b(McBatchSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t u;
    const McVol &d = mc_resolve(s, vols, u);
    mc::clip_unit(d, u, smem);
}

// Kernel pair (per-volume, batched) of pass ph of a plan, and its LDS bytes.
static KPair phase_kernels(const mclahe_plan_s *p, const McVol &v, int ph, size_t &lds)
{
    const int dt = p->in_dt;
    const bool ahr = p->mode == MC_AHR;
    lds = pass_lds(p, v, ph);
    switch (ph) {
    case 0:
        if (ahr)
            return dt == MC_U8 ? mc_pick_hist_u8(true, true, 0, false)
                 : dt == MC_U16 ? mc_pick_hist_u16(true, true, 0) : mc_pick_hist_f32(true, true, 0);
        return dt == MC_U8 ? mc_pick_range_u8() : dt == MC_U16 ? mc_pick_range_u16() : mc_pick_range_f32();
    case 1:
        return dt == MC_U8 ? mc_pick_hist_u8(ahr, false, v.hPeel, v.vhist != 0)
             : dt == MC_U16 ? mc_pick_hist_u16(ahr, false, v.hPeel) : mc_pick_hist_f32(ahr, false, v.hPeel);
    case 2:
        return KPair{(KFn)k_clip, (KFnB)k_clip_b, MC_T};
    default:
        return dt == MC_U8 ? mc_pick_map_u8(p->D, ahr, v.path)
             : dt == MC_U16 ? mc_pick_map_u16(p->D, ahr, v.path) : mc_pick_map_f32(p->D, ahr, v.path);
    }
}

static mclahe_status launch(KFn f, uint32_t grid, int threads, size_t lds, hipStream_t st, const McVol &v)
{
    if (grid == 0) return MCLAHE_SUCCESS;
    hipLaunchKernelGGL(f, dim3(grid), dim3(threads), lds, st, v);
    HIPCHK(hipGetLastError());
    return MCLAHE_SUCCESS;
}

static mclahe_status run_plain(const mclahe_plan_s *p, const McVol &v, hipStream_t st,
                               hipEvent_t *ev = nullptr)
{
    mclahe_status s;
    for (int ph = 0; ph < MC_PHASES; ++ph) {
        if (ev) HIPCHK(hipEventRecord(ev[ph], st));
        size_t lds = 0;
        const KPair k = phase_kernels(p, v, ph, lds);
        if ((s = launch(k.plain, mc_phase_units(v, ph), k.threads, lds, st, v))) return s;
    }
    if (ev) HIPCHK(hipEventRecord(ev[MC_PHASES], st));
    return MCLAHE_SUCCESS;
}

// ---------------------------------------------------------------- chunked --
// Out-of-core runs: the volume stays in host memory and passes through the
// device in slabs of whole kernel layers along axis 0 (the paper's outlook
// on chunked processing of data that does not fit in memory).  Histograms,
// clipping and LUTs of a kernel layer need only that layer's rows, so slab j
// histograms kernel layers [kA, kB).  An interpolation cell straddles two
// kernel layers, so slab j maps cell layers [kA - 1, kB - 1) with the LUTs of
// layers [kA - 1, kB - 1]: the last LUT layer of slab j - 1 is kept as a
// one-layer halo.  The global range (GHR) is one streamed min/max pass over
// all slabs first; its partials stay on the device and every histogram unit
// reduces them, exactly as in a whole-volume run.  Each launch runs the same
// kernels on the same work units as mclahe_run, with axis-0 windows, so the
// output is bit-identical.
struct ChunkGeom {
    int L = 0, n0 = 0;
    std::vector<int> kA, kB, cA, cB;          // per slab: kernel and cell layers
    std::vector<int64_t> hr0, hr1, mr0, mr1;  // per slab: rows read (hist, map)
    std::vector<int64_t> base;                // per slab: first row held in its buffer
    std::vector<int64_t> rr0, rr1;            // range blocks (GHR)
    std::vector<uint32_t> rparts;             // partials of each range block
    uint32_t range_parts = 0;
    int64_t row_elems = 1, layer_kernels = 1, cols_per_layer = 1, mcols_per_layer = 1;
    int64_t max_rows = 0, max_out_rows = 0;
    uint64_t o_in, o_in2, o_out, o_out2, o_part, o_rpart, o_hist, o_clipped, o_range, o_scale, o_lut, o_mrange, o_mscale,
        total;
};

static uint32_t range_units(int64_t nvox)
{
    return (uint32_t)std::min<int64_t>(1024, std::max<int64_t>(1, nvox / (MC_T * 64)));
}

static mclahe_status chunk_geom(const mclahe_plan_s *p, int L, ChunkGeom &g)
{
    if (p->D < 2) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "chunked runs need at least 2 dimensions");
    const McAxis &a0 = p->ax[0];
    if (L < 1) return fail(MCLAHE_ERROR_INVALID_VALUE, "slab_layers must be >= 1");
    L = std::min(L, a0.n);
    g = ChunkGeom();
    g.L = L;
    g.n0 = a0.n;
    for (int i = 1; i < p->D; ++i) {
        g.row_elems *= p->shape[i];
        g.layer_kernels *= p->ax[i].n;
        if (i < p->D - 1) {
            g.cols_per_layer *= p->ax[i].n;
            g.mcols_per_layer *= p->ax[i].n - 1;
        }
    }
    const int ns = (a0.n + L - 1) / L;
    for (int j = 0; j < ns; ++j) {
        const int kA = j * L, kB = std::min(kA + L, a0.n);
        int64_t lo = INT64_MAX, hi = -1;
        for (int k = kA; k < kB; ++k) {
            const McBox b = mc_kernel_box(a0, k);
            lo = std::min<int64_t>(lo, b.lo);
            hi = std::max<int64_t>(hi, b.hi);
        }
        const int cA = j == 0 ? 0 : kA - 1, cB = j == ns - 1 ? a0.n - 1 : kB - 1;
        int64_t mlo = 0, mhi = 0;
        if (cB > cA) {
            int l0, h0, l1, h1;
            mc_cell_range(a0, cA, l0, h0);
            mc_cell_range(a0, cB - 1, l1, h1);
            mlo = l0;
            mhi = h1;
        }
        g.kA.push_back(kA);
        g.kB.push_back(kB);
        g.cA.push_back(cA);
        g.cB.push_back(cB);
        g.hr0.push_back(lo);
        g.hr1.push_back(hi);
        g.mr0.push_back(mlo);
        g.mr1.push_back(mhi);
        // the slab's buffer holds rows [min(mlo, lo), hi): the map's halo
        // rows (the second half of the previous kernel layer) and the
        // histogram rows; the map rows lie inside
        const int64_t b0 = cB > cA ? std::min(mlo, lo) : lo;
        g.base.push_back(b0);
        g.max_rows = std::max(g.max_rows, hi - b0);
        g.max_out_rows = std::max(g.max_out_rows, mhi - mlo);
    }
    if (p->mode == MC_GHR && !p->has_ur) {
        for (int64_t r = 0; r < a0.s; r += g.max_rows) {
            const int64_t r1 = std::min<int64_t>(a0.s, r + g.max_rows);
            g.rr0.push_back(r);
            g.rr1.push_back(r1);
            const uint32_t u = range_units((r1 - r) * g.row_elems);
            g.rparts.push_back(u);
            g.range_parts += u;
        }
    }
    // partials of the slab's histogram units, for either decomposition (a
    // slab buffer is vector-aligned whenever vector loads are possible, but
    // the scalar one is sized too)
    int64_t nhg = 0;
    for (const McVol *v : {&p->v, &p->v1})
        nhg = std::max<int64_t>(nhg, (int64_t)L * g.cols_per_layer * v->hS * v->hCr * v->hG);
    const int64_t nk = (int64_t)L * g.layer_kernels;
    uint64_t o = 0;
    g.o_in = o;   // two slab buffers, used alternately (halo rows pass from one to the next)
    o = align256(o + (uint64_t)g.max_rows * g.row_elems * esize(p->in_dt));
    g.o_in2 = o;
    o = align256(o + (uint64_t)g.max_rows * g.row_elems * esize(p->in_dt));
    g.o_out = o;
    o = align256(o + (uint64_t)g.max_out_rows * g.row_elems * esize(p->out_dt));
    g.o_out2 = o;
    o = align256(o + (uint64_t)g.max_out_rows * g.row_elems * esize(p->out_dt));
    g.o_part = o;
    o = align256(o + (uint64_t)nhg * p->nb * 4);
    g.o_rpart = o;
    o = align256(o + (p->mode == MC_GHR ? (uint64_t)std::max<uint32_t>(g.range_parts, 1) * 2
                                        : (uint64_t)nhg * 2) * 4);
    g.o_hist = o;
    o = align256(o + (uint64_t)nk * p->nb * 4);
    g.o_clipped = o;
    o = align256(o + (uint64_t)nk * p->nb * 8);
    g.o_range = o;
    o = align256(o + 2 * 4);
    g.o_scale = o;
    o = align256(o + 4);
    g.o_lut = o;   // (L + 1) layers: the halo layer, then the slab's layers
    o = align256(o + (uint64_t)(L + 1) * g.layer_kernels * p->nb * 4);
    g.o_mrange = o;
    g.o_mscale = o;
    if (p->mode == MC_AHR) {
        o = align256(o + (uint64_t)(L + 1) * g.layer_kernels * 2 * 4);
        g.o_mscale = o;
        o = align256(o + (uint64_t)(L + 1) * g.layer_kernels * 4);
    }
    g.total = o;
    return MCLAHE_SUCCESS;
}

// Copy streams and events of chunked runs, per device, created on first use
// and kept for the life of the process (default priority).  Host-to-device
// copies run on `h2d`, device-to-host copies on `d2h`, kernels on the
// caller's stream; events order the three.  Runs on one device are
// serialised by `mu` while they are enqueued.
struct ChunkStreams {
    hipStream_t h2d = nullptr, d2h = nullptr;
    hipEvent_t in_ready[2], in_free[2], out_ready[2], out_free[2];
    std::mutex mu;
};
static std::mutex g_chunk_mu;
static std::map<int, ChunkStreams *> g_chunk_streams;

static mclahe_status chunk_streams(ChunkStreams *&cs)
{
    int dev = 0;
    HIPCHK(hipGetDevice(&dev));
    std::lock_guard<std::mutex> lk(g_chunk_mu);
    auto it = g_chunk_streams.find(dev);
    if (it != g_chunk_streams.end()) {
        cs = it->second;
        return MCLAHE_SUCCESS;
    }
    ChunkStreams *c = new ChunkStreams();
    HIPCHK(hipStreamCreateWithFlags(&c->h2d, hipStreamNonBlocking));
    HIPCHK(hipStreamCreateWithFlags(&c->d2h, hipStreamNonBlocking));
    for (int i = 0; i < 2; ++i) {
        HIPCHK(hipEventCreateWithFlags(&c->in_ready[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->in_free[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->out_ready[i], hipEventDisableTiming));
        HIPCHK(hipEventCreateWithFlags(&c->out_free[i], hipEventDisableTiming));
    }
    g_chunk_streams[dev] = c;
    cs = c;
    return MCLAHE_SUCCESS;
}

// Two input slab buffers and two output buffers alternate: the upload of
// the next slab (and of the next range block) overlaps the kernels of the
// current one, and the download of a slab's output overlaps both.
static mclahe_status run_chunked(const mclahe_plan_s *p, const ChunkGeom &g, const char *h_in, char *h_out,
                                 char *ws, hipStream_t st)
{
    mclahe_status s;
    ChunkStreams *cs = nullptr;
    if ((s = chunk_streams(cs))) return s;
    std::lock_guard<std::mutex> run_lock(cs->mu);
    const size_t es_in = esize(p->in_dt), es_out = esize(p->out_dt);
    const size_t row_in = (size_t)g.row_elems * es_in, row_out = (size_t)g.row_elems * es_out;
    char *inbuf[2] = {ws + g.o_in, ws + g.o_in2};
    char *outbuf[2] = {ws + g.o_out, ws + g.o_out2};
    bool in_used[2] = {false, false}, out_used[2] = {false, false};
    const size_t layer_lut = (size_t)g.layer_kernels * p->nb;   // floats per LUT layer
    float *lutb = (float *)(ws + g.o_lut);
    float *mrange = (float *)(ws + g.o_mrange), *mscale = (float *)(ws + g.o_mscale);
    const bool ahr = p->mode == MC_AHR;
    size_t lds = 0;
    int nin = 0;   // input buffer uses so far (range blocks, then slabs)

    // upload rows [r0, r1) of the host volume to input buffer X at row
    // offset `at` (rows before `at` were filled otherwise), on the copy stream
    auto upload = [&](int X, int64_t at, int64_t r0, int64_t r1) -> mclahe_status {
        if (in_used[X]) HIPCHK(hipStreamWaitEvent(cs->h2d, cs->in_free[X], 0));
        HIPCHK(hipMemcpyAsync(inbuf[X] + (size_t)at * row_in, h_in + (size_t)r0 * row_in,
                              (size_t)(r1 - r0) * row_in, hipMemcpyHostToDevice, cs->h2d));
        HIPCHK(hipEventRecord(cs->in_ready[X], cs->h2d));
        HIPCHK(hipStreamWaitEvent(st, cs->in_ready[X], 0));
        return MCLAHE_SUCCESS;
    };

    // 1. global range: one streamed min/max pass (partials stay on the device)
    uint32_t rp = 0;
    for (size_t b = 0; b < g.rr0.size(); ++b, ++nin) {
        const int X = nin & 1;
        if ((s = upload(X, 0, g.rr0[b], g.rr1[b]))) return s;
        McVol v = p->v;
        v.in = mc_gp(inbuf[X]);
        v.nvox = (g.rr1[b] - g.rr0[b]) * g.row_elems;
        v.n_range_wu = g.rparts[b];
        v.rpart = mc_gp((float *)(ws + g.o_rpart) + 2 * (size_t)rp);

        const KPair k = phase_kernels(p, v, 0, lds);
        if ((s = launch(k.plain, v.n_range_wu, k.threads, lds, st, v))) return s;
        HIPCHK(hipEventRecord(cs->in_free[X], st));
        in_used[X] = true;
        rp += g.rparts[b];
    }

    // 2. slabs: histograms, clip/CDF/LUT, interpolation
    int prevX = -1;
    for (size_t j = 0; j < g.kA.size(); ++j, ++nin) {
        const int kA = g.kA[j], kB = g.kB[j], nl = kB - kA;
        const int X = nin & 1, Y = (int)(j & 1);
        if (j > 0) {
            // the previous slab's last LUT layer becomes the halo layer 0
            const int last = g.kB[j - 1] - g.kA[j - 1];
            HIPCHK(hipMemcpyAsync(lutb, lutb + (size_t)last * layer_lut, layer_lut * 4,
                                  hipMemcpyDeviceToDevice, st));
            if (ahr) {
                HIPCHK(hipMemcpyAsync(mrange, mrange + (size_t)last * g.layer_kernels * 2,
                                      (size_t)g.layer_kernels * 2 * 4, hipMemcpyDeviceToDevice, st));
                HIPCHK(hipMemcpyAsync(mscale, mscale + (size_t)last * g.layer_kernels,
                                      (size_t)g.layer_kernels * 4, hipMemcpyDeviceToDevice, st));
            }
        }
        // slab buffer: halo rows [base, hr0) from the previous slab's buffer
        // (device to device, on the copy stream after that buffer's upload),
        // then the new rows [hr0, hr1) from the host
        char *cur = inbuf[X];
        const int64_t base = g.base[j];
        if (g.hr0[j] > base) {
            if (in_used[X]) HIPCHK(hipStreamWaitEvent(cs->h2d, cs->in_free[X], 0));
            in_used[X] = false;   // waited above
            HIPCHK(hipMemcpyAsync(cur, inbuf[prevX] + (size_t)(base - g.base[j - 1]) * row_in,
                                  (size_t)(g.hr0[j] - base) * row_in, hipMemcpyDeviceToDevice, cs->h2d));
        }
        if ((s = upload(X, g.hr0[j] - base, g.hr0[j], g.hr1[j]))) return s;
        // the slab's buffers index global rows; vector loads need them aligned
        const char *sin = cur - (size_t)base * row_in;
        char *sout = outbuf[Y] - (size_t)g.mr0[j] * row_out;
        McVol v = vec_aligned(p, sin, sout) ? p->v : p->v1;
        v.vhist = 0;   // the global range is known before the slabs: bin histograms
        v.wk0 = kA;
        v.n_hist_wu = (uint32_t)((int64_t)nl * g.cols_per_layer * v.hS * v.hCr);
        v.n_clip_wu = (uint32_t)((int64_t)nl * g.layer_kernels);
        v.n_range_wu = g.range_parts;
        v.in = mc_gp(sin);
        v.out = nullptr;
        v.part = mc_gp((uint32_t *)(ws + g.o_part));
        v.rpart = mc_gp((float *)(ws + g.o_rpart));
        v.hist = mc_gp((uint32_t *)(ws + g.o_hist));
        v.clipped = mc_gp((unsigned long long *)(ws + g.o_clipped));
        v.lut = mc_gp(lutb + layer_lut);                     // slab layers after the halo
        if (ahr) {
            v.range = mc_gp(mrange + (size_t)g.layer_kernels * 2);
            v.scale = mc_gp(mscale + g.layer_kernels);
        } else {
            v.range = mc_gp((float *)(ws + g.o_range));
            v.scale = mc_gp((float *)(ws + g.o_scale));
        }
        for (int ph = 0; ph < 3; ++ph) {
            const KPair k = phase_kernels(p, v, ph, lds);
            if (ph == 0 && !ahr) continue;            // GHR range done above
            if ((s = launch(k.plain, mc_phase_units(v, ph), k.threads, lds, st, v))) return s;
        }
        const int cA = g.cA[j], cB = g.cB[j];
        if (cB > cA) {
            const int64_t mrows = g.mr1[j] - g.mr0[j];
            McVol m = v;
            m.wc0 = cA;
            m.n_map_wu = (uint32_t)((int64_t)(cB - cA) * g.mcols_per_layer * v.mS * v.mU);
            m.in = mc_gp(sin);
            m.out = mc_gp(sout);
            // LUT layer 0 of the buffer is global kernel layer kA - 1
            m.lut = mc_gp(lutb - (int64_t)(kA - 1) * (int64_t)layer_lut);
            if (ahr) {
                m.range = mc_gp(mrange - (int64_t)(kA - 1) * g.layer_kernels * 2);
                m.scale = mc_gp(mscale - (int64_t)(kA - 1) * g.layer_kernels);
            }
            if (out_used[Y]) HIPCHK(hipStreamWaitEvent(st, cs->out_free[Y], 0));
            const KPair k = phase_kernels(p, m, 3, lds);
            if ((s = launch(k.plain, m.n_map_wu, k.threads, lds, st, m))) return s;
            HIPCHK(hipEventRecord(cs->out_ready[Y], st));
            HIPCHK(hipStreamWaitEvent(cs->d2h, cs->out_ready[Y], 0));
            HIPCHK(hipMemcpyAsync(h_out + (size_t)g.mr0[j] * row_out, outbuf[Y], (size_t)mrows * row_out,
                                  hipMemcpyDeviceToHost, cs->d2h));
            HIPCHK(hipEventRecord(cs->out_free[Y], cs->d2h));
            out_used[Y] = true;
        }
        HIPCHK(hipEventRecord(cs->in_free[X], st));
        in_used[X] = true;
        prevX = X;
    }
    // the caller's stream completes only after the last download
    for (int Y = 0; Y < 2; ++Y)
        if (out_used[Y]) HIPCHK(hipStreamWaitEvent(st, cs->out_free[Y], 0));
    for (int X = 0; X < 2; ++X)
        if (in_used[X]) HIPCHK(hipStreamWaitEvent(cs->h2d, cs->in_free[X], 0));
    return MCLAHE_SUCCESS;
}

struct mclahe_timer_s {
    std::vector<hipEvent_t> ev;   // 5 per run
    int max_runs = 0, runs = 0;
};

// Batched workspace: [descriptor table | per-volume workspaces...].  The
// table (header, launch records, index arrays, volume descriptors) is written
// by one stream-ordered copy per call; the per-volume workspaces are laid out
// as for mclahe_run.  Launch grouping depends only on the plans.
struct BatchLaunch {
    int phase;
    KFnB fn;
    KFnB group;                   // clip pass: the volumes' histogram class
    int threads;
    size_t lds;
    std::vector<uint32_t> vols;   // volume indices
    std::vector<uint32_t> pre;    // unit prefix sums
};

struct BatchLayout {
    std::vector<mclahe_plan_s> view;   // the plans with their batched decomposition
    uint64_t o_table, o_recs, o_idx, o_vols, o_phdr, o_pre, o_q, o_first, total;
    std::vector<uint64_t> vol_off;
    std::vector<BatchLaunch> launches;
    uint32_t n_idx = 0;
};

// ins / outs (may be NULL: sizing only) pick each volume's decomposition:
// vector loads for 16-byte aligned buffers, scalar loads otherwise.  Sizes
// and offsets do not depend on them.
static mclahe_status batch_layout(int n, const mclahe_plan_t *plans, const void *const *ins,
                                  void *const *outs, BatchLayout &L)
{
    if (n < 1 || !plans) return fail(MCLAHE_ERROR_INVALID_VALUE, "batched call needs n >= 1 plans");
    for (int i = 0; i < n; ++i)
        if (!plans[i]) return fail(MCLAHE_ERROR_INVALID_VALUE, "plan %d is NULL", i);
    L.view.resize(n);
    for (int i = 0; i < n; ++i) {
        batch_view(plans[i], L.view[i]);
        if (ins && outs && !vec_aligned(&L.view[i], ins[i], outs[i])) L.view[i].v = L.view[i].v1;
    }
    // group the volumes of each pass by kernel class
    L.launches.clear();
    for (int ph = 0; ph < MC_PHASES; ++ph) {
        const size_t first = L.launches.size();
        for (int i = 0; i < n; ++i) {
            const mclahe_plan_s *p = &L.view[i];
            const uint32_t units = mc_phase_units(p->v, ph);
            if (!units) continue;
            size_t lds = 0;
            const KPair k = phase_kernels(p, p->v, ph, lds);
            // the clip pass has one kernel for every volume; it is split by
            // the volumes' histogram class so that each class forms a chain
            // of launches that does not wait for the others (graph replay)
            KFnB group = nullptr;
            if (ph == 2) {
                size_t lh = 0;
                group = phase_kernels(p, p->v, 1, lh).batch;
            }
            BatchLaunch *bl = nullptr;
            for (size_t j = first; j < L.launches.size(); ++j)
                if (L.launches[j].fn == k.batch && L.launches[j].group == group) bl = &L.launches[j];
            if (!bl) {
                L.launches.push_back(BatchLaunch{ph, k.batch, group, k.threads, 0, {}, {0}});
                bl = &L.launches.back();
            }
            bl->lds = std::max(bl->lds, lds);
            bl->vols.push_back((uint32_t)i);
            bl->pre.push_back(bl->pre.back() + units);
        }
        // Work-groups are dispatched in index order as the chip frees room:
        // put the volumes with the largest units first, so that the launch
        // ends on small units instead of waiting for a few large ones that
        // started last (longest-first list scheduling).
        for (size_t j = first; j < L.launches.size(); ++j) {
            BatchLaunch &bl = L.launches[j];
            auto per_unit = [&](uint32_t i) {
                return (double)L.view[i].nvox / (double)mc_phase_units(L.view[i].v, ph);
            };
            std::stable_sort(bl.vols.begin(), bl.vols.end(),
                             [&](uint32_t a, uint32_t b) { return per_unit(a) > per_unit(b); });
            bl.pre.assign(1, 0u);
            for (uint32_t i : bl.vols) bl.pre.push_back(bl.pre.back() + mc_phase_units(L.view[i].v, ph));
        }
    }
    L.n_idx = 0;
    for (auto &bl : L.launches) L.n_idx += (uint32_t)(bl.vols.size() + bl.pre.size());
    uint64_t o = 0;
    L.o_table = o;
    o = align256(o + sizeof(McBatchHdr));
    L.o_recs = o;
    o = align256(o + L.launches.size() * sizeof(McLaunchRec));
    L.o_idx = o;
    o = align256(o + (uint64_t)L.n_idx * 4);
    L.o_vols = o;
    o = align256(o + (uint64_t)n * sizeof(McVol));
    // the persistent launch's table: header, unit prefix sums per pass, and
    // the run's words (ticket head, abort word, completion counters)
    L.o_phdr = o;
    o = align256(o + sizeof(McPersistHdr));
    L.o_pre = o;
    o = align256(o + (uint64_t)MC_PHASES * (n + 1) * 4);
    L.o_q = o;
    o = align256(o + (uint64_t)mc_persist_words((uint32_t)n) * 4);
    L.o_first = o;
    L.vol_off.resize(n);
    for (int i = 0; i < n; ++i) {
        L.vol_off[i] = o;
        o = align256(o + L.view[i].total);
    }
    L.total = o;
    return MCLAHE_SUCCESS;
}

// Host image of the table region [o_table, o_first).
// Volume i's workspace is vol_ws[i].
static void fill_table(int n, const mclahe_plan_t *plans, const void *const *ins, void *const *outs,
                       char *const *vol_ws, const BatchLayout &L, std::vector<char> &img)
{
    img.assign(L.o_first - L.o_table, 0);
    McBatchHdr *h = (McBatchHdr *)img.data();
    McLaunchRec *recs = (McLaunchRec *)(img.data() + L.o_recs);
    uint32_t *idx = (uint32_t *)(img.data() + L.o_idx);
    McVol *vols = (McVol *)(img.data() + L.o_vols);
    for (int i = 0; i < n; ++i) bind(&L.view[i], vols[i], ins[i], outs[i], vol_ws[i]);
    h->nvol = (uint32_t)n;
    h->nlaunch = (uint32_t)L.launches.size();
    h->o_persist = (uint32_t)(L.o_phdr - L.o_table);
    {   // persistent launch: tickets in pass-major, batch order
        McPersistHdr *ph = (McPersistHdr *)(img.data() + L.o_phdr);
        uint32_t *pre = (uint32_t *)(img.data() + L.o_pre);
        ph->nvol = (uint32_t)n;
        ph->max_spins = kPersistSpins;
        ph->abort_at = MC_NO_TICKET;
        uint32_t t = 0;
        for (int p = 0; p < MC_PHASES; ++p) {
            ph->phase_start[p] = t;
            uint32_t *pp = pre + p * (n + 1);
            pp[0] = 0;
            for (int i = 0; i < n; ++i) pp[i + 1] = pp[i] + mc_phase_units(L.view[i].v, p);
            t += pp[n];
        }
        ph->phase_start[MC_PHASES] = t;
        ph->total = t;
    }
    uint32_t k = 0;
    for (size_t j = 0; j < L.launches.size(); ++j) {
        const BatchLaunch &bl = L.launches[j];
        McLaunchRec &r = recs[j];
        r.phase = (uint32_t)bl.phase;
        r.n = (uint32_t)bl.vols.size();
        r.list = k;
        for (uint32_t v : bl.vols) idx[k++] = v;
        r.pre = k;
        for (uint32_t u : bl.pre) idx[k++] = u;
        r.units = bl.pre.back();
    }
}

// A batch signature (table address and the grid of every launch) seen for the
// first time is launched directly; when it repeats, its launches are captured
// in a graph,
// kept in a small LRU cache with a ring of pinned host images of the
// descriptor table (a slot is reused only after the copy that read it ran).
struct GraphEntry {
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    std::vector<char *> host;
    std::vector<hipEvent_t> ev;
    std::vector<bool> used;
    int next = 0;
    size_t bytes = 0;
    uint64_t last_use = 0;
};

static std::mutex g_graph_mu;
static std::map<std::string, GraphEntry *> g_graphs;
static std::set<std::string> g_seen;      // batch signatures launched directly once
static uint64_t g_tick = 0;
static const size_t kGraphCacheMax = 16;

static void destroy_graph(GraphEntry *g)
{
    for (size_t r = 0; r < g->ev.size(); ++r) {
        if (g->used[r]) (void)hipEventSynchronize(g->ev[r]);
        (void)hipEventDestroy(g->ev[r]);
    }
    for (char *h : g->host) (void)hipHostFree(h);
    if (g->exec) (void)hipGraphExecDestroy(g->exec);
    if (g->graph) (void)hipGraphDestroy(g->graph);
    delete g;
}

// Pinned staging ring for descriptor tables of directly launched batches: a
// slot is reused (or grown) only after the copy that read it has completed.
struct StageSlot {
    char *host = nullptr;
    size_t cap = 0;
    hipEvent_t ev = nullptr;
    bool used = false;
};
static StageSlot g_stage[8];
static int g_stage_next = 0;

static mclahe_status stage_table(const std::vector<char> &img, void *dst, hipStream_t st)
{
    StageSlot &sl = g_stage[g_stage_next];
    g_stage_next = (g_stage_next + 1) % 8;
    if (!sl.ev) HIPCHK(hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming));
    if (sl.used) HIPCHK(hipEventSynchronize(sl.ev));
    if (sl.cap < img.size()) {
        // grow the whole ring at once (pinned allocations are slow): later
        // calls of this size or smaller then never allocate
        size_t cap = size_t(64) << 10;
        while (cap < img.size()) cap <<= 1;
        for (StageSlot &o : g_stage) {
            if (o.cap >= cap) continue;
            if (o.used) HIPCHK(hipEventSynchronize(o.ev));
            if (o.host) HIPCHK(hipHostFree(o.host));
            o.host = nullptr;
            o.cap = 0;
            o.used = false;
            HIPCHK(hipHostMalloc((void **)&o.host, cap, hipHostMallocDefault));
            o.cap = cap;
        }
    }
    memcpy(sl.host, img.data(), img.size());
    HIPCHK(hipMemcpyAsync(dst, sl.host, img.size(), hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(sl.ev, st));
    sl.used = true;
    return MCLAHE_SUCCESS;
}

// Graph: a launch depends on the launches that last ran one of its volumes
// (each volume's passes run in order; volumes share no workspace or output),
// so the chains of different kernel classes overlap.
static mclahe_status build_graph(GraphEntry *g, const BatchLayout &L, const std::vector<char> &img, char *table)
{
    HIPCHK(hipGraphCreate(&g->graph, 0));
    const McLaunchRec *recs = (const McLaunchRec *)(img.data() + L.o_recs);
    const uint32_t *idx_dev = (const uint32_t *)(table + L.o_idx);
    const McVol *vols_dev = (const McVol *)(table + L.o_vols);
    std::vector<hipGraphNode_t> nodes(L.launches.size());
    std::vector<int> last(L.view.size(), -1);   // latest launch of each volume
    for (size_t j = 0; j < L.launches.size(); ++j) {
        const BatchLaunch &bl = L.launches[j];
        std::vector<int> dep;
        for (uint32_t v : bl.vols)
            if (last[v] >= 0) dep.push_back(last[v]);
        std::sort(dep.begin(), dep.end());
        dep.erase(std::unique(dep.begin(), dep.end()), dep.end());
        std::vector<hipGraphNode_t> prev;
        for (int q : dep) prev.push_back(nodes[q]);
        if (bl.lds > 64 * 1024)
            HIPCHK(hipFuncSetAttribute((const void *)bl.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bl.lds));
        McBatchSrc src;
        src.vols = vols_dev;
        src.list = idx_dev + recs[j].list;
        src.pre = idx_dev + recs[j].pre;
        src.n = recs[j].n;
        src.pad_ = 0;
        const McVol *vols_arg = vols_dev;
        void *args[] = {&src, &vols_arg};
        hipKernelNodeParams kp = {};
        kp.func = (void *)bl.fn;
        kp.gridDim = dim3(recs[j].units);
        kp.blockDim = dim3(bl.threads);
        kp.sharedMemBytes = (unsigned)bl.lds;
        kp.kernelParams = args;
        hipGraphNode_t node;
        HIPCHK(hipGraphAddKernelNode(&node, g->graph, prev.empty() ? nullptr : prev.data(), prev.size(), &kp));
        nodes[j] = node;
        for (uint32_t v : bl.vols) last[v] = (int)j;
    }
    HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
    return MCLAHE_SUCCESS;
}

// --------------------------------------------------------------- autotune --
static std::mutex g_tune_mu;
static std::map<std::string, mclahe_tuning> g_tune_cache;
static bool g_tune_loaded = false;

static std::string plan_key(const mclahe_plan_s *p)
{
    std::string k = "D" + std::to_string(p->D);
    for (int i = 0; i < p->D; ++i) k += "_" + std::to_string(p->shape[i]) + "x" + std::to_string(p->ks[i]);
    k += "_n" + std::to_string(p->nb) + "_m" + std::to_string(p->mode) + "_i" + std::to_string(p->in_dt) +
         "_o" + std::to_string(p->out_dt) + "_u" + std::to_string(p->has_ur);
    return k;
}

static void tune_cache_load()
{
    if (g_tune_loaded) return;
    g_tune_loaded = true;
    const char *f = getenv("MCLAHE_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "r");
    if (!fp) return;
    char key[512];
    mclahe_tuning t;
    while (fscanf(fp, "%511s %d %d %d %d %d %d", key, &t.hist_rows_split, &t.hist_copies, &t.hist_peel,
                  &t.map_rows_split, &t.map_group, &t.map_unit_chunks) == 7)
        g_tune_cache[key] = t;
    fclose(fp);
}

static void tune_cache_store(const std::string &key, const mclahe_tuning &t)
{
    g_tune_cache[key] = t;
    const char *f = getenv("MCLAHE_TUNE_CACHE");
    if (!f) return;
    FILE *fp = fopen(f, "a");
    if (!fp) return;
    fprintf(fp, "%s %d %d %d %d %d %d\n", key.c_str(), t.hist_rows_split, t.hist_copies, t.hist_peel,
            t.map_rows_split, t.map_group, t.map_unit_chunks);
    fclose(fp);
}

static std::vector<mclahe_tuning> tune_candidates(const mclahe_plan_s *p)
{
    std::vector<mclahe_tuning> c;
    const McVol &v = p->v;
    const int hcr = v.hCr, mcr = v.mCr;
    for (int R : {1, 2, 4})
        for (int peel : {1, 2})
            for (int f : {1, 2, 4}) {
                mclahe_tuning t = {};
                t.hist_copies = R;
                t.hist_peel = peel;
                t.hist_rows_split = std::max(1, hcr * f / 2);
                t.map_rows_split = mcr;
                t.map_group = v.mG;
                c.push_back(t);
            }
    return c;
}

// ---------------------------------------------------------------- C ABI --
extern "C" {

const char *mclahe_version(void) { return "0.1.0"; }

const char *mclahe_status_string(mclahe_status s)
{
    switch (s) {
    case MCLAHE_SUCCESS: return "MCLAHE_SUCCESS";
    case MCLAHE_ERROR_INVALID_VALUE: return "MCLAHE_ERROR_INVALID_VALUE";
    case MCLAHE_ERROR_NOT_SUPPORTED: return "MCLAHE_ERROR_NOT_SUPPORTED";
    case MCLAHE_ERROR_OUT_OF_MEMORY: return "MCLAHE_ERROR_OUT_OF_MEMORY";
    case MCLAHE_ERROR_WORKSPACE: return "MCLAHE_ERROR_WORKSPACE";
    case MCLAHE_ERROR_HIP: return "MCLAHE_ERROR_HIP";
    }
    return "MCLAHE_UNKNOWN_STATUS";
}

const char *mclahe_last_error(void) { return g_err.c_str(); }

mclahe_status mclahe_plan(mclahe_plan_t *plan, int ndim, const int64_t *shape, const int64_t *kernel_size,
                          int n_bins, double clip_limit, mclahe_range_mode mode, const float *user_range,
                          mclahe_dtype in_dtype, mclahe_dtype out_dtype)
{
    g_err.clear();
    if (!plan) return fail(MCLAHE_ERROR_INVALID_VALUE, "plan pointer is NULL");
    *plan = nullptr;
    if (ndim < 1 || ndim > MC_MAXD) return fail(MCLAHE_ERROR_INVALID_VALUE, "ndim must be in 1..8 (got %d)", ndim);
    if (!shape || !kernel_size) return fail(MCLAHE_ERROR_INVALID_VALUE, "shape/kernel_size is NULL");
    if (n_bins < 2 || n_bins > 8192) return fail(MCLAHE_ERROR_INVALID_VALUE, "n_bins must be in 2..8192 (got %d)", n_bins);
    if (!(clip_limit >= 0.0) || std::isinf(clip_limit))
        return fail(MCLAHE_ERROR_INVALID_VALUE, "clip_limit must be finite and >= 0");
    if (mode != MCLAHE_RANGE_GLOBAL && mode != MCLAHE_RANGE_KERNEL)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "unknown range mode %d", (int)mode);
    if (in_dtype < MCLAHE_U8 || in_dtype > MCLAHE_F32 || out_dtype < MCLAHE_U8 || out_dtype > MCLAHE_F32)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "unknown dtype");
    if (user_range) {
        if (mode != MCLAHE_RANGE_GLOBAL)
            return fail(MCLAHE_ERROR_INVALID_VALUE, "a user range is only valid with the global range mode");
        if (!std::isfinite(user_range[0]) || !std::isfinite(user_range[1]) || !(user_range[0] < user_range[1]))
            return fail(MCLAHE_ERROR_INVALID_VALUE, "user range must be finite with lo < hi");
    }
    mclahe_plan_s *p = new (std::nothrow) mclahe_plan_s();
    if (!p) return fail(MCLAHE_ERROR_OUT_OF_MEMORY, "host allocation failed");
    p->D = ndim;
    p->nb = n_bins;
    p->clip = clip_limit;
    p->mode = mode;
    p->has_ur = user_range != nullptr;
    p->ur[0] = user_range ? user_range[0] : 0.f;
    p->ur[1] = user_range ? user_range[1] : 0.f;
    p->in_dt = in_dtype;
    p->out_dt = out_dtype;
    p->nvox = 1;
    p->nker = 1;
    p->K = 1;
    p->ncells = 1;
    for (int i = 0; i < ndim; ++i) {
        const int64_t s = shape[i], b = kernel_size[i];
        if (s < 1 || s > INT32_MAX / 4) {
            delete p;
            return fail(MCLAHE_ERROR_INVALID_VALUE, "shape[%d]=%lld out of range", i, (long long)s);
        }
        if (b < 1 || b > s) {
            delete p;
            return fail(MCLAHE_ERROR_INVALID_VALUE, "kernel_size[%d]=%lld must be in 1..shape[%d]=%lld", i,
                        (long long)b, i, (long long)s);
        }
        p->shape[i] = s;
        p->ks[i] = b;
        const int64_t pad = 2 * b - 1 - ((s - 1) % b);   // Eq. 1
        p->ax[i].s = (int32_t)s;
        p->ax[i].b = (int32_t)b;
        p->ax[i].p0 = (int32_t)(pad / 2);                // Eq. 2
        p->ax[i].p1 = (int32_t)((pad + 1) / 2);
        p->ax[i].n = (int32_t)((s + pad) / b);
        p->ax[i].cw = (int32_t)(b - 1);                   // centre at k*b + (b-1)/2
        p->nvox *= s;
        p->nker *= p->ax[i].n;
        p->K *= b;
        p->ncells *= p->ax[i].n - 1;
        if (p->nvox >= ((int64_t)1 << 40) || p->nker >= ((int64_t)1 << 31)) {
            delete p;
            return fail(MCLAHE_ERROR_NOT_SUPPORTED, "volume too large");
        }
    }
    for (int i = ndim; i < MC_MAXD; ++i) {
        p->ax[i] = McAxis{1, 1, 0, 1, 2, 0};
        p->shape[i] = p->ks[i] = 1;
    }
    if (p->K >= ((int64_t)1 << 32)) {
        delete p;
        return fail(MCLAHE_ERROR_NOT_SUPPORTED, "kernel voxel count must be < 2^32");
    }
    int64_t st = 1;
    for (int i = ndim - 1; i >= 0; --i) {
        p->stride[i] = st;
        st *= p->shape[i];
    }
    for (int i = ndim; i < MC_MAXD; ++i) p->stride[i] = 0;
    p->clipC = clip_count(clip_limit, p->K);
    memset(&p->tune, 0, sizeof p->tune);
    memset(&p->btune, 0, sizeof p->btune);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_load();
        auto it = g_tune_cache.find(plan_key(p));
        if (it != g_tune_cache.end()) p->tune = it->second;
        auto ib = g_tune_cache.find("B" + plan_key(p));
        if (ib != g_tune_cache.end()) p->btune = ib->second;
    }
    mclahe_status s = derive(p);
    if (s != MCLAHE_SUCCESS && (p->tune.hist_rows_split || p->tune.map_rows_split || p->btune.hist_rows_split ||
                                p->btune.map_rows_split)) {
        memset(&p->tune, 0, sizeof p->tune);
        memset(&p->btune, 0, sizeof p->btune);
        s = derive(p);
    }
    if (s != MCLAHE_SUCCESS) {
        delete p;
        return s;
    }
    *plan = p;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_destroy(mclahe_plan_t plan)
{
    delete plan;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_geometry(mclahe_plan_t p, mclahe_geometry *g)
{
    if (!p || !g) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    memset(g, 0, sizeof *g);
    g->ndim = p->D;
    for (int i = 0; i < p->D; ++i) {
        g->pad[i] = p->ax[i].p0 + p->ax[i].p1;
        g->pad0[i] = p->ax[i].p0;
        g->pad1[i] = p->ax[i].p1;
        g->n_kernels_axis[i] = p->ax[i].n;
    }
    g->n_kernels = p->nker;
    g->kernel_voxels = p->K;
    g->clip_count = p->clipC;
    g->n_voxels = p->nvox;
    g->n_cells = p->ncells;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_get_tuning(mclahe_plan_t p, mclahe_tuning *t)
{
    if (!p || !t) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    t->hist_rows_split = p->v.hCr;
    t->hist_copies = p->v.hR;
    t->hist_peel = p->v.hPeel + 1;
    t->map_rows_split = p->v.mCr;
    t->map_unit_chunks = p->v.mK;
    t->map_group = p->v.mG;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_set_tuning(mclahe_plan_t p, const mclahe_tuning *t)
{
    if (!p || !t) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (t->hist_rows_split < 0 || t->map_rows_split < 0 || t->map_group < 0 || t->map_unit_chunks < 0 ||
        t->hist_peel < 0 ||
        t->hist_peel > 3 || t->hist_copies < 0)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "tuning fields must be >= 0 (hist_peel <= 3)");
    const mclahe_tuning old = p->tune;
    p->tune = *t;
    mclahe_status s = derive(p);
    if (s != MCLAHE_SUCCESS) {
        const std::string msg = g_err;
        p->tune = old;
        derive(p);
        g_err = msg;
    }
    return s;
}

mclahe_status mclahe_plan_get_batch_tuning(mclahe_plan_t p, mclahe_tuning *t)
{
    if (!p || !t) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    t->hist_rows_split = p->bv.hCr;
    t->hist_copies = p->bv.hR;
    t->hist_peel = p->bv.hPeel + 1;
    t->map_rows_split = p->bv.mCr;
    t->map_unit_chunks = p->bv.mK;
    t->map_group = p->bv.mG;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_set_batch_tuning(mclahe_plan_t p, const mclahe_tuning *t)
{
    if (!p || !t) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (t->hist_rows_split < 0 || t->map_rows_split < 0 || t->map_group < 0 || t->map_unit_chunks < 0 ||
        t->hist_peel < 0 || t->hist_peel > 3 || t->hist_copies < 0)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "tuning fields must be >= 0 (hist_peel <= 3)");
    const mclahe_tuning old = p->btune;
    p->btune = *t;
    mclahe_status s = derive(p);
    if (s != MCLAHE_SUCCESS) {
        const std::string msg = g_err;
        p->btune = old;
        derive(p);
        g_err = msg;
    }
    return s;
}

mclahe_status mclahe_plan_get_variant(mclahe_plan_t p, mclahe_variant *v)
{
    if (!p || !v) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    v->redistribution = p->redist;
    v->rounds = p->rounds;
    v->centre = p->centre_half;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_plan_set_variant(mclahe_plan_t p, const mclahe_variant *v)
{
    if (!p || !v) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (v->redistribution < MCLAHE_REDIST_EQUAL || v->redistribution > MCLAHE_REDIST_INTEGER)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "unknown redistribution %d", v->redistribution);
    if (v->centre != MCLAHE_CENTRE_MIDDLE && v->centre != MCLAHE_CENTRE_HALF)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "unknown centre convention %d", v->centre);
    const int rounds = v->redistribution == MCLAHE_REDIST_REPEATED ? v->rounds : 1;
    if (rounds < 1 || rounds > 8) return fail(MCLAHE_ERROR_INVALID_VALUE, "rounds must be in 1..8");
    // the last round counts in units of 1/n^rounds: n^rounds * K must fit
    long double units = (long double)p->K;
    for (int r = 0; r < rounds; ++r) units *= (long double)p->nb;
    if (units >= 9.0e18L)
        return fail(MCLAHE_ERROR_NOT_SUPPORTED, "n_bins^rounds * kernel voxels must stay below 2^63");
    p->redist = v->redistribution;
    p->rounds = rounds;
    p->centre_half = v->centre;
    for (int i = 0; i < p->D; ++i) p->ax[i].cw = (int32_t)(v->centre ? 2 * (p->ks[i] / 2) : p->ks[i] - 1);
    return derive(p);
}

mclahe_status mclahe_workspace_size(mclahe_plan_t p, size_t *bytes)
{
    if (!p || !bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    *bytes = p->total;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_workspace_layout(mclahe_plan_t p, mclahe_layout *l)
{
    if (!p || !l) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    l->hist = p->o_hist;
    l->clipped = p->o_clipped;
    l->lut = p->o_lut;
    l->range = p->o_range;
    l->scale = p->o_scale;
    l->total = p->total;
    return MCLAHE_SUCCESS;
}

static mclahe_status check_run_args(const mclahe_plan_s *p, const void *in, void *out, void *ws,
                                    size_t wsb, size_t need)
{
    if (!p) return fail(MCLAHE_ERROR_INVALID_VALUE, "plan is NULL");
    if (!in || !out) return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output pointer is NULL");
    if (((uintptr_t)in % esize(p->in_dt)) || ((uintptr_t)out % esize(p->out_dt)))
        return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output not aligned to the element size");
    if (in == out && esize(p->in_dt) != esize(p->out_dt))
        return fail(MCLAHE_ERROR_INVALID_VALUE, "in-place operation needs equal element sizes");
    if (!ws || ((uintptr_t)ws % 256)) return fail(MCLAHE_ERROR_WORKSPACE, "workspace NULL or not 256-byte aligned");
    if (wsb < need)
        return fail(MCLAHE_ERROR_WORKSPACE, "workspace too small: %zu < %zu bytes", wsb, need);
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run(mclahe_plan_t p, const void *d_in, void *d_out, void *d_ws, size_t wsb, void *stream)
{
    g_err.clear();
    mclahe_status s = check_run_args(p, d_in, d_out, d_ws, wsb, p ? p->total : 0);
    if (s) return s;
    McVol v;
    bind(p, v, d_in, d_out, (char *)d_ws);
    return run_plain(p, v, (hipStream_t)stream);
}

// ------------------------------------------------- run with the metrics --
// Workspace: the plan's own, then one metric record per interpolation unit
// (either decomposition), then the metric passes' own arrays.
static uint64_t met_parts_off(const mclahe_plan_s *p) { return align256(p->total); }
static uint64_t met_tail_off(const mclahe_plan_s *p)
{
    const uint64_t nu = std::max(p->v.n_map_wu, p->v1.n_map_wu);
    return met_parts_off(p) + align256(nu * sizeof(McMetPart));
}

mclahe_status mclahe_run_metrics_workspace_size(mclahe_plan_t p, int n_bins, size_t *bytes)
{
    if (!p || !bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (n_bins < 2 || n_bins > 8192) return fail(MCLAHE_ERROR_INVALID_VALUE, "metric n_bins must be in [2, 8192]");
    *bytes = met_tail_off(p) + mc_metrics_tail_ws(p->nvox, n_bins, (int)std::max(p->v.n_map_wu, p->v1.n_map_wu));
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_metrics(mclahe_plan_t p, const void *d_in, void *d_out, void *d_ws, size_t wsb,
                                 int n_bins, double peak, mclahe_metrics_result *d_result, uint64_t *d_hist,
                                 void *stream)
{
    g_err.clear();
    size_t need = 0;
    mclahe_status s = mclahe_run_metrics_workspace_size(p, n_bins, &need);
    if (s) return s;
    if (!d_result) return fail(MCLAHE_ERROR_INVALID_VALUE, "result pointer is NULL");
    if (!(peak > 0.0) || !std::isfinite(peak)) return fail(MCLAHE_ERROR_INVALID_VALUE, "peak must be positive and finite");
    if (d_in == d_out) return fail(MCLAHE_ERROR_INVALID_VALUE, "metrics need the input after the run: not in place");
    if ((s = check_run_args(p, d_in, d_out, d_ws, wsb, need))) return s;
    McVol v;
    bind(p, v, d_in, d_out, (char *)d_ws);
    v.met = mc_gp((McMetPart *)((char *)d_ws + met_parts_off(p)));
    hipStream_t st = (hipStream_t)stream;
    for (int ph = 0; ph < 3; ++ph) {
        size_t lds = 0;
        const KPair k = phase_kernels(p, v, ph, lds);
        if ((s = launch(k.plain, mc_phase_units(v, ph), k.threads, lds, st, v))) return s;
    }
    size_t lds = 0;
    const KPair k = phase_kernels(p, v, 3, lds);
    const int dt = p->in_dt, ahr = p->mode == MC_AHR;
    const KFn fm = dt == MC_U8 ? mc_pick_map_met_u8(p->D, ahr, v.path)
                 : dt == MC_U16 ? mc_pick_map_met_u16(p->D, ahr, v.path) : mc_pick_map_met_f32(p->D, ahr, v.path);
    if ((s = launch(fm, v.n_map_wu, k.threads, std::max<size_t>(lds, 256), st, v))) return s;
    return mc_metrics_tail(d_in, p->in_dt, d_out, p->out_dt, p->nvox, n_bins, peak, v.met, (int)v.n_map_wu,
                           d_result, d_hist, (char *)d_ws + met_tail_off(p), st);
}

// --------------------------------------------- smoothing, then the method --
// Workspace: the plan's own, the Gaussian's intermediate volume, then the
// (min, max) pairs of the Gaussian's last pass.
static mclahe_status smooth_layout(const mclahe_plan_s *p, const double *sigma, double truncate, uint64_t &o_gws,
                                   uint64_t &gws, uint64_t &o_mm, int64_t &nmm, uint64_t &total)
{
    size_t g = 0;
    mclahe_status s = mclahe_gaussian_workspace_size(p->D, p->shape, sigma, &g);
    if (s) return s;
    nmm = 0;
    if (p->mode == MC_GHR && !p->has_ur && truncate > 0.0 && std::isfinite(truncate))
        nmm = mc_gaussian_mm_parts(p->D, p->shape, sigma, truncate);
    o_gws = align256(p->total);
    gws = g;
    o_mm = align256(o_gws + g);
    total = align256(o_mm + (uint64_t)nmm * 8);
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_smoothed_workspace_size(mclahe_plan_t p, const double *sigma, double truncate, size_t *bytes)
{
    if (!p || !sigma || !bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    uint64_t o_gws, gws, o_mm, total;
    int64_t nmm;
    mclahe_status s = smooth_layout(p, sigma, truncate, o_gws, gws, o_mm, nmm, total);
    if (s) return s;
    *bytes = total;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_smoothed(mclahe_plan_t p, const void *d_in, mclahe_dtype in_dtype, const double *sigma,
                                  double truncate, float *d_smooth, void *d_out, void *d_ws, size_t wsb, void *stream)
{
    g_err.clear();
    if (!p || !sigma) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (p->in_dt != MC_F32) return fail(MCLAHE_ERROR_INVALID_VALUE, "the plan must take float input (the smoothed volume)");
    uint64_t o_gws, gws, o_mm, total;
    int64_t nmm;
    mclahe_status s = smooth_layout(p, sigma, truncate, o_gws, gws, o_mm, nmm, total);
    if (s) return s;
    if ((s = check_run_args(p, d_smooth, d_out, d_ws, wsb, total))) return s;
    if ((const void *)d_smooth == d_in) return fail(MCLAHE_ERROR_INVALID_VALUE, "the smoothed volume must not overlap the input");
    hipStream_t st = (hipStream_t)stream;
    char *ws = (char *)d_ws;
    float *mm = nmm > 0 ? (float *)(ws + o_mm) : nullptr;
    if ((s = mc_gaussian_run(d_in, in_dtype, p->D, p->shape, sigma, truncate, d_smooth, gws ? ws + o_gws : nullptr, gws,
                             mm, st)))
        return s;
    McVol v;
    bind(p, v, d_smooth, d_out, ws);
    int ph0 = 0;
    if (mm) {   // the smoothing pass took the global range: fold its pairs into the range partials
        if ((s = mc_minmax_reduce(mm, nmm, v.rpart, v.n_range_wu, st))) return s;
        ph0 = 1;
    }
    for (int ph = ph0; ph < MC_PHASES; ++ph) {
        size_t lds = 0;
        const KPair k = phase_kernels(p, v, ph, lds);
        if ((s = launch(k.plain, mc_phase_units(v, ph), k.threads, lds, st, v))) return s;
    }
    return MCLAHE_SUCCESS;
}

// ------------------------------------------------------ no-allocation run --
// A file-scope device array serves as the workspace of mclahe_run_noalloc.
// In host code its name is only a stand-in: the device address of each GPU's
// copy comes from hipGetSymbolAddress, taken once per device with that
// device current, and only that address is handed to kernels.  Every pass
// writes all it hands to the next one (range partials, histogram partials,
// per-kernel arrays), so the array never needs clearing between calls.
static __device__ __align__(256) unsigned char scratch[MCLAHE_NOALLOC_SCRATCH_BYTES];

static const int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static char *g_scratch_ptr[kMaxDevices];   // per device, NULL until set up

static mclahe_status scratch_ptr(char *&ptr)
{
    int dev = -1;
    HIPCHK(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "device %d beyond %d", dev, kMaxDevices);
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *a = nullptr;
        HIPCHK(hipGetSymbolAddress(&a, HIP_SYMBOL(scratch)));
        if (!a || ((uintptr_t)a % 256)) return fail(MCLAHE_ERROR_HIP, "scratch array address %p unusable", a);
        g_scratch_ptr[dev] = (char *)a;
    }
    ptr = g_scratch_ptr[dev];
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_noalloc(mclahe_plan_t p, const void *d_in, void *d_out, void *stream)
{
    g_err.clear();
    if (!p) return fail(MCLAHE_ERROR_INVALID_VALUE, "plan is NULL");
    if (p->total > MCLAHE_NOALLOC_SCRATCH_BYTES)
        return fail(MCLAHE_ERROR_WORKSPACE, "plan needs %llu workspace bytes, more than the %llu of the static scratch",
                    (unsigned long long)p->total, (unsigned long long)MCLAHE_NOALLOC_SCRATCH_BYTES);
    char *ws = nullptr;
    mclahe_status s = scratch_ptr(ws);
    if (s) return s;
    s = check_run_args(p, d_in, d_out, ws, MCLAHE_NOALLOC_SCRATCH_BYTES, p->total);
    if (s) return s;
    McVol v;
    bind(p, v, d_in, d_out, ws);
    return run_plain(p, v, (hipStream_t)stream);
}

mclahe_status mclahe_timer_create(mclahe_timer_t *timer, int max_runs)
{
    if (!timer || max_runs < 1 || max_runs > 100000)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "timer needs 1..100000 runs");
    *timer = nullptr;
    mclahe_timer_s *t = new (std::nothrow) mclahe_timer_s();
    if (!t) return fail(MCLAHE_ERROR_OUT_OF_MEMORY, "host allocation failed");
    t->max_runs = max_runs;
    t->ev.resize((size_t)max_runs * 5, nullptr);
    for (auto &e : t->ev) {
        if (hipEventCreate(&e) != hipSuccess) {
            for (auto &f : t->ev)
                if (f) (void)hipEventDestroy(f);
            delete t;
            return fail(MCLAHE_ERROR_HIP, "hipEventCreate failed");
        }
    }
    *timer = t;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_timer_destroy(mclahe_timer_t t)
{
    if (!t) return MCLAHE_SUCCESS;
    for (auto &e : t->ev) (void)hipEventDestroy(e);
    delete t;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_timer_reset(mclahe_timer_t t)
{
    if (!t) return fail(MCLAHE_ERROR_INVALID_VALUE, "timer is NULL");
    t->runs = 0;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_timed(mclahe_plan_t p, const void *d_in, void *d_out, void *d_ws, size_t wsb,
                               void *stream, mclahe_timer_t t)
{
    g_err.clear();
    if (!t) return fail(MCLAHE_ERROR_INVALID_VALUE, "timer is NULL");
    if (t->runs >= t->max_runs) return fail(MCLAHE_ERROR_INVALID_VALUE, "timer is full (%d runs)", t->max_runs);
    mclahe_status s = check_run_args(p, d_in, d_out, d_ws, wsb, p ? p->total : 0);
    if (s) return s;
    McVol v;
    bind(p, v, d_in, d_out, (char *)d_ws);
    s = run_plain(p, v, (hipStream_t)stream, &t->ev[(size_t)t->runs * 5]);
    if (s == MCLAHE_SUCCESS) t->runs++;
    return s;
}

mclahe_status mclahe_timer_read(mclahe_timer_t t, float *pass_ms, int *runs)
{
    if (!t || !pass_ms || !runs) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    *runs = t->runs;
    for (int k = 0; k < 4; ++k) pass_ms[k] = 0.f;
    if (t->runs == 0) return MCLAHE_SUCCESS;
    HIPCHK(hipEventSynchronize(t->ev[(size_t)(t->runs - 1) * 5 + 4]));
    for (int r = 0; r < t->runs; ++r)
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, t->ev[(size_t)r * 5 + k], t->ev[(size_t)r * 5 + k + 1]));
            pass_ms[k] += ms / t->runs;
        }
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_batched_workspace_size(int n, const mclahe_plan_t *plans, size_t *bytes)
{
    if (!bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, nullptr, nullptr, L);
    if (s) return s;
    *bytes = L.total;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_batched_workspace_offsets(int n, const mclahe_plan_t *plans, uint64_t *offsets)
{
    if (!offsets) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, nullptr, nullptr, L);
    if (s) return s;
    for (int i = 0; i < n; ++i) offsets[i] = L.vol_off[i];
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_batched_table_size(int n, const mclahe_plan_t *plans, size_t *bytes)
{
    if (!bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, nullptr, nullptr, L);
    if (s) return s;
    *bytes = L.o_first - L.o_table;
    return MCLAHE_SUCCESS;
}

static void vol_ws_in_place(int n, char *ws, const BatchLayout &L, std::vector<char *> &vws)
{
    vws.resize(n);
    for (int i = 0; i < n; ++i) vws[i] = ws + L.vol_off[i];
}

mclahe_status mclahe_batched_table(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                   void *const *d_out, void *d_ws, void *host_image, size_t image_bytes,
                                   size_t *needed)
{
    g_err.clear();
    if (!d_in || !d_out || !needed) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, d_in, d_out, L);
    if (s) return s;
    std::vector<char *> vws;
    vol_ws_in_place(n, (char *)d_ws, L, vws);
    std::vector<char> img;
    fill_table(n, plans, d_in, d_out, vws.data(), L, img);
    *needed = img.size();
    if (host_image) memcpy(host_image, img.data(), std::min(image_bytes, img.size()));
    return MCLAHE_SUCCESS;
}

// Upload the table image to `table` and run the launches of L on st: directly
// on the first sight of the batch's structure, from a cached graph after.
// The key holds everything a graph bakes in: the table address and, per
// launch, kernel, volume count, grid, block and LDS size.  Everything else a
// kernel reads comes from the table uploaded before each replay.
static mclahe_status batched_direct(const BatchLayout &L, const std::vector<char> &img, char *table,
                                    hipStream_t st)
{
    mclahe_status s;
    if ((s = stage_table(img, table, st))) return s;
    const McLaunchRec *recs = (const McLaunchRec *)(img.data() + L.o_recs);
    const uint32_t *idx_dev = (const uint32_t *)(table + L.o_idx);
    const McVol *vols_dev = (const McVol *)(table + L.o_vols);
    for (size_t j = 0; j < L.launches.size(); ++j) {
        const BatchLaunch &bl = L.launches[j];
        if (bl.lds > 64 * 1024)
            HIPCHK(hipFuncSetAttribute((const void *)bl.fn, hipFuncAttributeMaxDynamicSharedMemorySize,
                                       (int)bl.lds));
        McBatchSrc src{vols_dev, idx_dev + recs[j].list, idx_dev + recs[j].pre, recs[j].n, 0};
        hipLaunchKernelGGL(bl.fn, dim3(recs[j].units), dim3(bl.threads), bl.lds, st, src, src.vols);
        HIPCHK(hipGetLastError());
    }
    return MCLAHE_SUCCESS;
}

static mclahe_status batched_launch(const BatchLayout &L, const std::vector<char> &img, char *table,
                                    hipStream_t st)
{
    mclahe_status s;
    const McLaunchRec *recs = (const McLaunchRec *)(img.data() + L.o_recs);
    std::string key = std::to_string((uintptr_t)table);
    for (size_t j = 0; j < L.launches.size(); ++j) {
        const BatchLaunch &bl = L.launches[j];
        char buf[96];
        snprintf(buf, sizeof buf, ":%zx/%u/%u/%d/%zu/", (size_t)(uintptr_t)bl.fn, recs[j].n, recs[j].units,
                 bl.threads, bl.lds);
        key += buf;
        // the graph's edges follow which volumes each launch runs
        for (uint32_t v : bl.vols) key += std::to_string(v) + ",";
    }
    std::lock_guard<std::mutex> lk(g_graph_mu);
    ++g_tick;
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        if (!g_seen.count(key)) {
            // first sight of this batch: direct launches, remember the signature
            if (g_seen.size() > 4096) g_seen.clear();
            g_seen.insert(key);
            return batched_direct(L, img, table, st);
        }
        // repeated batch: capture it as a graph (bounded cache, LRU eviction)
        if (g_graphs.size() >= kGraphCacheMax) {
            auto victim = g_graphs.begin();
            for (auto e = g_graphs.begin(); e != g_graphs.end(); ++e)
                if (e->second->last_use < victim->second->last_use) victim = e;
            destroy_graph(victim->second);
            g_graphs.erase(victim);
        }
        GraphEntry *g = new GraphEntry();
        g->bytes = img.size();
        for (int r = 0; r < 4; ++r) {
            char *hb = nullptr;
            hipEvent_t e = nullptr;
            if (hipHostMalloc((void **)&hb, g->bytes, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                if (hb) (void)hipHostFree(hb);
                destroy_graph(g);
                return fail(MCLAHE_ERROR_HIP, "pinned staging buffer or event creation failed");
            }
            g->host.push_back(hb);
            g->ev.push_back(e);
            g->used.push_back(false);
        }
        s = build_graph(g, L, img, table);
        if (s) {
            destroy_graph(g);
            return s;
        }
        it = g_graphs.emplace(key, g).first;
    }
    GraphEntry *g = it->second;
    g->last_use = g_tick;
    const int slot = g->next;
    g->next = (g->next + 1) % (int)g->host.size();
    if (g->used[slot]) HIPCHK(hipEventSynchronize(g->ev[slot]));
    memcpy(g->host[slot], img.data(), g->bytes);
    HIPCHK(hipMemcpyAsync(table, g->host[slot], g->bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(g->ev[slot], st));
    g->used[slot] = true;
    HIPCHK(hipGraphLaunch(g->exec, st));
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_batched(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                 void *const *d_out, void *d_ws, size_t wsb, void *stream)
{
    g_err.clear();
    if (!d_in || !d_out) return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output arrays are NULL");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, d_in, d_out, L);
    if (s) return s;
    for (int i = 0; i < n; ++i) {
        s = check_run_args(plans[i], d_in[i], d_out[i], d_ws, wsb, L.total);
        if (s) return fail(s, "volume %d: %s", i, g_err.c_str());
    }
    char *ws = (char *)d_ws;
    std::vector<char *> vws;
    vol_ws_in_place(n, ws, L, vws);
    std::vector<char> img;
    fill_table(n, plans, d_in, d_out, vws.data(), L, img);
    return batched_launch(L, img, ws + L.o_table, (hipStream_t)stream);
}

// ------------------------------------------------ persistent batched run --
// Grid and LDS of the persistent launch of a batch: as many work-groups as
// fit the chip at once (no more than the tickets), and the LDS of the
// largest unit of any pass of any volume.
static mclahe_status persist_shape(const BatchLayout &L, const std::vector<char> &img, uint32_t &grid, size_t &lds)
{
    lds = 0;
    for (const mclahe_plan_s &q : L.view)
        for (int ph = 0; ph < MC_PHASES; ++ph) lds = std::max(lds, pass_lds(&q, q.v, ph));
    lds = std::max<size_t>(lds, 16);
    int dev = 0, cus = 0, per_cu = 0;
    HIPCHK(hipGetDevice(&dev));
    HIPCHK(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
    // (the kernel's own static LDS is a few words on top)
    if (lds + 256 > 64 * 1024)
        HIPCHK(hipFuncSetAttribute(mc_persist_fn(), hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds));
    HIPCHK(hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, mc_persist_fn(), MC_T, lds));
    if (per_cu < 1) return fail(MCLAHE_ERROR_NOT_SUPPORTED, "persistent kernel does not fit a compute unit");
    const uint32_t total = ((const McPersistHdr *)(img.data() + L.o_phdr))->total;
    grid = (uint32_t)std::min<int64_t>((int64_t)cus * per_cu, std::max<uint32_t>(total, 1));
    return MCLAHE_SUCCESS;
}

static void persist_args(const BatchLayout &L, char *table, McPersistSrc &src, uint32_t *&q, uint32_t &nq)
{
    src.hdr = (const McPersistHdr *)(table + L.o_phdr);
    src.pre = (const uint32_t *)(table + L.o_pre);
    src.vols = (const McVol *)(table + L.o_vols);
    src.q = (uint32_t *)(table + L.o_q);
    q = src.q;
    nq = mc_persist_words((uint32_t)L.view.size());
}

// One persistent run: the table upload, a kernel clearing the run's words,
// the persistent kernel.  A batch seen before is replayed from a graph of
// those two kernels (same cache as the per-pass batched graphs).
static mclahe_status persistent_launch(const BatchLayout &L, const std::vector<char> &img, char *table,
                                       hipStream_t st)
{
    mclahe_status s;
    uint32_t grid = 0;
    size_t lds = 0;
    if ((s = persist_shape(L, img, grid, lds))) return s;
    McPersistSrc src;
    uint32_t *q = nullptr, nq = 0;
    persist_args(L, table, src, q, nq);
    const uint32_t rgrid = (nq + MC_T - 1) / MC_T;
    char buf[128];
    snprintf(buf, sizeof buf, "P%zx/%u/%u/%zu/%zu", (size_t)(uintptr_t)table, grid,
             ((const McPersistHdr *)(img.data() + L.o_phdr))->total, lds, L.view.size());
    const std::string key(buf);
    std::lock_guard<std::mutex> lk(g_graph_mu);
    ++g_tick;
    auto it = g_graphs.find(key);
    if (it == g_graphs.end()) {
        if (!g_seen.count(key)) {
            if (g_seen.size() > 4096) g_seen.clear();
            g_seen.insert(key);
            if ((s = stage_table(img, table, st))) return s;
            hipLaunchKernelGGL((void (*)(uint32_t *, uint32_t))mc_persist_reset_fn(), dim3(rgrid), dim3(MC_T), 0, st,
                               q, nq);
            hipLaunchKernelGGL((void (*)(McPersistSrc, const McVol *))mc_persist_fn(), dim3(grid), dim3(MC_T), lds, st,
                               src, src.vols);
            HIPCHK(hipGetLastError());
            return MCLAHE_SUCCESS;
        }
        if (g_graphs.size() >= kGraphCacheMax) {
            auto victim = g_graphs.begin();
            for (auto e = g_graphs.begin(); e != g_graphs.end(); ++e)
                if (e->second->last_use < victim->second->last_use) victim = e;
            destroy_graph(victim->second);
            g_graphs.erase(victim);
        }
        GraphEntry *g = new GraphEntry();
        g->bytes = img.size();
        for (int r = 0; r < 4; ++r) {
            char *hb = nullptr;
            hipEvent_t e = nullptr;
            if (hipHostMalloc((void **)&hb, g->bytes, hipHostMallocDefault) != hipSuccess ||
                hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
                if (hb) (void)hipHostFree(hb);
                destroy_graph(g);
                return fail(MCLAHE_ERROR_HIP, "pinned staging buffer or event creation failed");
            }
            g->host.push_back(hb);
            g->ev.push_back(e);
            g->used.push_back(false);
        }
        auto build = [&]() -> mclahe_status {
            HIPCHK(hipGraphCreate(&g->graph, 0));
            hipKernelNodeParams kr = {};
            void *rargs[] = {&q, &nq};
            kr.func = (void *)mc_persist_reset_fn();
            kr.gridDim = dim3(rgrid);
            kr.blockDim = dim3(MC_T);
            kr.sharedMemBytes = 0;
            kr.kernelParams = rargs;
            hipGraphNode_t nr, np;
            HIPCHK(hipGraphAddKernelNode(&nr, g->graph, nullptr, 0, &kr));
            hipKernelNodeParams kp = {};
            const McVol *vols_arg = src.vols;
            void *pargs[] = {&src, &vols_arg};
            kp.func = (void *)mc_persist_fn();
            kp.gridDim = dim3(grid);
            kp.blockDim = dim3(MC_T);
            kp.sharedMemBytes = (unsigned)lds;
            kp.kernelParams = pargs;
            HIPCHK(hipGraphAddKernelNode(&np, g->graph, &nr, 1, &kp));
            HIPCHK(hipGraphInstantiate(&g->exec, g->graph, nullptr, nullptr, 0));
            return MCLAHE_SUCCESS;
        };
        if ((s = build())) {
            destroy_graph(g);
            return s;
        }
        it = g_graphs.emplace(key, g).first;
    }
    GraphEntry *g = it->second;
    g->last_use = g_tick;
    const int slot = g->next;
    g->next = (g->next + 1) % (int)g->host.size();
    if (g->used[slot]) HIPCHK(hipEventSynchronize(g->ev[slot]));
    memcpy(g->host[slot], img.data(), g->bytes);
    HIPCHK(hipMemcpyAsync(table, g->host[slot], g->bytes, hipMemcpyHostToDevice, st));
    HIPCHK(hipEventRecord(g->ev[slot], st));
    g->used[slot] = true;
    HIPCHK(hipGraphLaunch(g->exec, st));
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_batched_persistent(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                            void *const *d_out, void *d_ws, size_t wsb,
                                            const mclahe_persistent_opts *opts, void *stream)
{
    g_err.clear();
    if (!d_in || !d_out) return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output arrays are NULL");
    if (opts && (opts->flags & ~MCLAHE_PERSIST_ABORT_TICKET))
        return fail(MCLAHE_ERROR_INVALID_VALUE, "unknown persistent-run flags 0x%x", opts->flags);
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, d_in, d_out, L);
    if (s) return s;
    for (int i = 0; i < n; ++i) {
        s = check_run_args(plans[i], d_in[i], d_out[i], d_ws, wsb, L.total);
        if (s) return fail(s, "volume %d: %s", i, g_err.c_str());
    }
    char *ws = (char *)d_ws;
    std::vector<char *> vws;
    vol_ws_in_place(n, ws, L, vws);
    std::vector<char> img;
    fill_table(n, plans, d_in, d_out, vws.data(), L, img);
    McPersistHdr *h = (McPersistHdr *)(img.data() + L.o_phdr);
    if (opts && opts->max_spins) h->max_spins = opts->max_spins;
    if (opts && (opts->flags & MCLAHE_PERSIST_ABORT_TICKET)) h->abort_at = opts->abort_ticket;
    return persistent_launch(L, img, ws + L.o_table, (hipStream_t)stream);
}

mclahe_status mclahe_persistent_status(int n, const mclahe_plan_t *plans, const void *d_ws, uint32_t *aborted,
                                       uint32_t *tickets, void *stream)
{
    g_err.clear();
    if (!d_ws || !aborted) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, nullptr, nullptr, L);
    if (s) return s;
    HIPCHK(hipStreamSynchronize((hipStream_t)stream));
    uint32_t w[2] = {0, 0};
    HIPCHK(hipMemcpy(w, (const char *)d_ws + L.o_table + L.o_q, sizeof w, hipMemcpyDeviceToHost));
    *aborted = w[MC_PQ_ABORT];
    if (tickets) *tickets = w[MC_PQ_HEAD];
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_batched_split(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                       void *const *d_out, void *const *d_ws, const size_t *ws_bytes,
                                       void *d_table, size_t table_bytes, void *stream)
{
    g_err.clear();
    if (!d_in || !d_out || !d_ws || !ws_bytes)
        return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output/workspace arrays are NULL");
    BatchLayout L;
    mclahe_status s = batch_layout(n, plans, d_in, d_out, L);
    if (s) return s;
    for (int i = 0; i < n; ++i) {
        s = check_run_args(plans[i], d_in[i], d_out[i], d_ws[i], ws_bytes[i], plans[i]->total);
        if (s) return fail(s, "volume %d: %s", i, g_err.c_str());
    }
    const size_t tb = L.o_first - L.o_table;
    if (!d_table || ((uintptr_t)d_table % 256))
        return fail(MCLAHE_ERROR_WORKSPACE, "descriptor table buffer NULL or not 256-byte aligned");
    if (table_bytes < tb)
        return fail(MCLAHE_ERROR_WORKSPACE, "descriptor table buffer too small: %zu < %zu bytes", table_bytes, tb);
    std::vector<char> img;
    fill_table(n, plans, d_in, d_out, (char *const *)d_ws, L, img);
    std::lock_guard<std::mutex> lk(g_graph_mu);      // the staging ring is shared
    return batched_direct(L, img, (char *)d_table, (hipStream_t)stream);
}

mclahe_status mclahe_chunked_workspace_size(mclahe_plan_t p, int slab_layers, size_t *bytes)
{
    if (!p || !bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    ChunkGeom g;
    mclahe_status s = chunk_geom(p, slab_layers, g);
    if (s) return s;
    *bytes = g.total;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_run_chunked(mclahe_plan_t p, const void *h_in, void *h_out, int slab_layers, void *d_ws,
                                 size_t wsb, void *stream)
{
    g_err.clear();
    if (!p || !h_in || !h_out || !d_ws) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    if (h_in == h_out) return fail(MCLAHE_ERROR_INVALID_VALUE, "chunked runs cannot work in place");
    ChunkGeom g;
    mclahe_status s = chunk_geom(p, slab_layers, g);
    if (s) return s;
    if ((uintptr_t)d_ws % 256) return fail(MCLAHE_ERROR_WORKSPACE, "workspace not 256-byte aligned");
    if (wsb < g.total) return fail(MCLAHE_ERROR_WORKSPACE, "workspace too small: %zu < %zu bytes", wsb,
                                   (size_t)g.total);
    return run_chunked(p, g, (const char *)h_in, (char *)h_out, (char *)d_ws, (hipStream_t)stream);
}

mclahe_status mclahe_autotune_workspace_size(mclahe_plan_t p, size_t *bytes)
{
    if (!p || !bytes) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument");
    const mclahe_tuning saved = p->tune;
    size_t mx = p->total;
    for (const mclahe_tuning &t : tune_candidates(p)) {
        mclahe_tuning tt = t;
        p->tune = tt;
        if (derive(p) == MCLAHE_SUCCESS) mx = std::max<size_t>(mx, p->total);
    }
    p->tune = saved;
    derive(p);
    *bytes = mx;
    return MCLAHE_SUCCESS;
}

mclahe_status mclahe_autotune(mclahe_plan_t p, const void *d_in, void *d_out, void *d_ws, size_t wsb,
                              void *stream)
{
    g_err.clear();
    size_t need = 0;
    mclahe_status s = mclahe_autotune_workspace_size(p, &need);
    if (s) return s;
    if ((s = check_run_args(p, d_in, d_out, d_ws, wsb, need))) return s;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    const mclahe_tuning saved = p->tune;
    auto time_cfg = [&](const mclahe_tuning &t, float &ms) -> mclahe_status {
        p->tune = t;
        mclahe_status r = derive(p);
        if (r) return r;
        McVol v;
        bind(p, v, d_in, d_out, (char *)d_ws);
        if ((r = run_plain(p, v, st))) return r;   // warm-up
        float best = 1e30f;
        for (int rep = 0; rep < 3; ++rep) {
            HIPCHK(hipEventRecord(e0, st));
            if ((r = run_plain(p, v, st))) return r;
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float t_ms = 0;
            HIPCHK(hipEventElapsedTime(&t_ms, e0, e1));
            best = std::min(best, t_ms);
        }
        ms = best;
        return MCLAHE_SUCCESS;
    };
    // histogram knobs first, then the interpolation knobs
    mclahe_tuning best_t = saved;
    float best_ms = 1e30f;
    for (const mclahe_tuning &t : tune_candidates(p)) {
        float ms;
        if (time_cfg(t, ms) == MCLAHE_SUCCESS && ms < best_ms) {
            best_ms = ms;
            best_t = t;
        }
    }
    p->tune = best_t;
    derive(p);
    const int ncl = p->ax[p->D - 1].n - 1;
    const int mcr0 = p->v.mCr;       // row split of the best histogram setting
    std::vector<int> groups = {1, 2, 4, ncl};
    for (int g : groups) {
        if (g < 1 || g > ncl) continue;
        for (int f : {1, 2, 4})
            for (int k : {0, 1, 2, 1 << 20}) {   // unit chunks: default, 1, 2, all
                mclahe_tuning t = best_t;
                t.map_group = g;
                t.map_rows_split = std::max(1, mcr0 * f / 2);
                t.map_unit_chunks = k == (1 << 20) ? t.map_rows_split : k;
                float ms;
                if (time_cfg(t, ms) == MCLAHE_SUCCESS && ms < best_ms) {
                    best_ms = ms;
                    best_t = t;
                }
            }
    }
    p->tune = best_t;
    derive(p);
    // store the effective settings
    mclahe_tuning eff;
    mclahe_plan_get_tuning(p, &eff);
    p->tune = eff;
    derive(p);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        tune_cache_store(plan_key(p), eff);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return MCLAHE_SUCCESS;
}

// Batched autotuning.  Volumes that run the same kernels form a class; the
// classes' launch chains overlap on the GPU, so a candidate is timed as the
// whole batch through mclahe_run_batched (graph replays).  Per class, in
// turn: the histogram row split (the default, or 2 or 4 times fewer, larger
// units) with 1 or 2 LDS replicas, then the interpolation row chunks per unit
// (half, the default, 2 or 4 times as many, or all).  Candidates never need
// more workspace than the defaults (fewer histogram units, fewer partials).
// The default is a candidate, and the result is kept only if it stays faster
// than the default when the two are timed again: tuned is never slower.
static std::string class_key(const mclahe_plan_s *p)
{
    return std::to_string(p->in_dt) + "/" + std::to_string(p->mode) + "/" + std::to_string(p->D) + "/" +
           std::to_string(p->bv.path);
}

// Workspace of the batch under the default batch tuning (the largest any
// candidate needs); the plans' batch tuning is left as it was.
mclahe_status mclahe_autotune_batched_workspace_size(int n, const mclahe_plan_t *plans, size_t *bytes)
{
    if (!bytes || n < 1 || !plans) return fail(MCLAHE_ERROR_INVALID_VALUE, "NULL argument or n < 1");
    for (int i = 0; i < n; ++i)
        if (!plans[i]) return fail(MCLAHE_ERROR_INVALID_VALUE, "plan %d is NULL", i);
    std::vector<mclahe_tuning> saved(n);
    mclahe_status s = MCLAHE_SUCCESS;
    for (int i = 0; i < n && !s; ++i) {
        saved[i] = plans[i]->btune;
        memset(&plans[i]->btune, 0, sizeof plans[i]->btune);
        s = derive(plans[i]);
    }
    if (!s) s = mclahe_batched_workspace_size(n, plans, bytes);
    for (int i = 0; i < n; ++i) {
        plans[i]->btune = saved[i];
        derive(plans[i]);
    }
    return s;
}

mclahe_status mclahe_autotune_batched(int n, const mclahe_plan_t *plans, const void *const *d_in,
                                      void *const *d_out, void *d_ws, size_t wsb, void *stream)
{
    g_err.clear();
    size_t need = 0;
    mclahe_status s = mclahe_autotune_batched_workspace_size(n, plans, &need);
    if (s) return s;
    if (!d_in || !d_out) return fail(MCLAHE_ERROR_INVALID_VALUE, "input/output arrays are NULL");
    if (wsb < need) return fail(MCLAHE_ERROR_WORKSPACE, "workspace too small: %zu < %zu bytes", wsb, need);
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    std::vector<mclahe_tuning> saved(n), def(n);
    for (int i = 0; i < n; ++i) saved[i] = plans[i]->btune;
    auto apply = [&](const std::vector<mclahe_tuning> &t) -> mclahe_status {
        for (int i = 0; i < n; ++i) {
            plans[i]->btune = t[i];
            mclahe_status r = derive(plans[i]);
            if (r) return r;
        }
        size_t w = 0;
        mclahe_status r = mclahe_batched_workspace_size(n, plans, &w);
        if (r) return r;
        return w <= wsb ? MCLAHE_SUCCESS : fail(MCLAHE_ERROR_WORKSPACE, "candidate needs more workspace");
    };
    auto time_batch = [&](float &best) -> mclahe_status {
        mclahe_status r;
        for (int w = 0; w < 3; ++w)   // direct, capture, first replay
            if ((r = mclahe_run_batched(n, plans, d_in, d_out, d_ws, wsb, stream))) return r;
        best = 1e30f;
        for (int rep = 0; rep < 5; ++rep) {
            HIPCHK(hipEventRecord(e0, st));
            if ((r = mclahe_run_batched(n, plans, d_in, d_out, d_ws, wsb, stream))) return r;
            HIPCHK(hipEventRecord(e1, st));
            HIPCHK(hipEventSynchronize(e1));
            float ms = 0.f;
            HIPCHK(hipEventElapsedTime(&ms, e0, e1));
            best = std::min(best, ms);
        }
        return MCLAHE_SUCCESS;
    };
    // defaults (batch tuning cleared) and the decomposition they give
    std::vector<McVol> dv(n);
    for (int i = 0; i < n; ++i) memset(&def[i], 0, sizeof def[i]);
    if ((s = apply(def))) goto out;
    for (int i = 0; i < n; ++i) dv[i] = plans[i]->bv;
    {
        std::map<std::string, std::vector<int>> cls;
        for (int i = 0; i < n; ++i) cls[class_key(plans[i])].push_back(i);
        std::vector<mclahe_tuning> cur = def;
        float cur_ms;
        if ((s = time_batch(cur_ms))) goto out;
        const float def_ms = cur_ms;
        for (auto &c : cls) {
            auto with = [&](int fh, int R, int fm2) {   // fm2: map chunks per unit x fm2 / 2; 0 = all
                std::vector<mclahe_tuning> t = cur;
                for (int i : c.second) {
                    const McVol &d = dv[i];
                    mclahe_tuning &u = t[i];
                    u.hist_rows_split = std::max(1, d.hCr / fh);
                    u.hist_copies = R;
                    u.map_rows_split = d.mCr;
                    u.map_group = d.mG;
                    u.map_unit_chunks = fm2 == 0 ? d.mCr : std::max(1, std::min(d.mCr, d.mK * fm2 / 2));
                }
                return t;
            };
            // start from the defaults (so that the map candidates keep the
            // default replicas when no histogram candidate wins)
            int bh = 1, bR = dv[c.second[0]].hR;
            for (int fh : {1, 2, 4})
                for (int R : {1, 2, 4}) {
                    std::vector<mclahe_tuning> t = with(fh, R, 2);
                    float ms;
                    if (apply(t) || time_batch(ms)) continue;
                    if (ms < cur_ms) {
                        cur_ms = ms;
                        cur = t;
                        bh = fh;
                        bR = R;
                    }
                }
            for (int fm2 : {1, 4, 8, 0}) {
                std::vector<mclahe_tuning> t = with(bh, bR, fm2);
                float ms;
                if (apply(t) || time_batch(ms)) continue;
                if (ms < cur_ms) {
                    cur_ms = ms;
                    cur = t;
                }
            }
        }
        // keep the result only if it beats the defaults again, both re-timed
        float d_ms = def_ms, t_ms = cur_ms;
        if ((s = apply(def)) || (s = time_batch(d_ms))) goto out;
        if ((s = apply(cur)) || (s = time_batch(t_ms))) goto out;
        if (!(t_ms < 0.99f * d_ms)) cur = def;
        if ((s = apply(cur))) goto out;
        std::lock_guard<std::mutex> lk(g_tune_mu);
        for (int i = 0; i < n; ++i) {
            mclahe_tuning eff;
            mclahe_plan_get_batch_tuning(plans[i], &eff);
            plans[i]->btune = cur[i].hist_rows_split ? eff : cur[i];
            derive(plans[i]);
            tune_cache_store("B" + plan_key(plans[i]), plans[i]->btune);
        }
    }
out:
    if (s) {   // leave the plans as they were
        for (int i = 0; i < n; ++i) {
            plans[i]->btune = saved[i];
            derive(plans[i]);
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return s;
}

}  // extern "C"
