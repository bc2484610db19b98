// Internal interface between the host runtime and the kernel translation
// units of the MCLAHE library.
#pragma once
#include "mc_desc.h"
#include "../../include/mclahe.h"

// Thread-local error message of the C ABI (set by a failing call).
mclahe_status mc_fail(mclahe_status s, const char *fmt, ...);
void mc_clear_error();

typedef void (*KFn)(McVol);         // per-volume kernel: one volume by value
typedef void (*KFnB)(McBatchSrc, const McVol *);   // batched twin: many volumes of one class
                                                   // (the descriptors again, as a restrict parameter)

struct KPair {
    KFn plain;
    KFnB batch;
    int threads;   // work-group size of both
};

KPair mc_pick_range_u8();
KPair mc_pick_range_u16();
KPair mc_pick_range_f32();
KPair mc_pick_hist_u8(bool ahr, bool ro, int peel, bool val);   // val: per-value slots
KPair mc_pick_hist_u16(bool ahr, bool ro, int peel);
KPair mc_pick_hist_f32(bool ahr, bool ro, int peel);
KPair mc_pick_map_u8(int D, bool ahr, int path);
KPair mc_pick_map_u16(int D, bool ahr, int path);
KPair mc_pick_map_f32(int D, bool ahr, int path);
// interpolation kernels that also write the contrast-metric partials
KFn mc_pick_map_met_u8(int D, bool ahr, int path);
KFn mc_pick_map_met_u16(int D, bool ahr, int path);
KFn mc_pick_map_met_f32(int D, bool ahr, int path);
// The contrast metrics of an input and its enhanced output from the partials
// the interpolation units wrote (nparts records): statistics, then one pass
// over both volumes for the centred sums and grey-level histograms, then the
// result.  mc_metrics_tail_ws: workspace bytes of those passes.
size_t mc_metrics_tail_ws(int64_t nvox, int n_bins, int nparts);
mclahe_status mc_metrics_tail(const void *x, int x_dt, const void *y, int y_dt, int64_t nvox, int n_bins,
                              double peak, const McMetPart *parts, int nparts, mclahe_metrics_result *res,
                              uint64_t *hist_out, char *ws, hipStream_t st);

// Pre-smoothing (mc_denoise.hip).  mc_gaussian_run is mclahe_gaussian that,
// given mm, also writes one (min, max) pair per work-group of its last pass
// when that pass is the fused last-two-axes one; mc_gaussian_mm_parts gives
// how many (0: the configuration's last pass writes none).
// mc_minmax_reduce folds n pairs into m pairs (m work-groups).
int64_t mc_gaussian_mm_parts(int ndim, const int64_t *shape, const double *sigma, double truncate);
mclahe_status mc_gaussian_run(const void *d_in, int in_dtype, int ndim, const int64_t *shape, const double *sigma,
                              double truncate, float *d_out, void *d_workspace, size_t workspace_bytes, float *mm,
                              hipStream_t st);
mclahe_status mc_minmax_reduce(const float *src, int64_t n, float *dst, uint32_t m, hipStream_t st);

// The persistent batched kernel (k_persist.hip): k_persist(McPersistSrc),
// and the kernel that clears a run's words, (uint32_t *q, uint32_t n).
const void *mc_persist_fn();
const void *mc_persist_reset_fn();
