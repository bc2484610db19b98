// Internal interface between the host runtime and the kernel translation
// units of the MCLAHE library.
#pragma once
#include "mc_desc.h"
#include "../../include/mclahe.h"

// Thread-local error message of the C ABI (set by a failing call).
mclahe_status mc_fail(mclahe_status s, const char *fmt, ...);
void mc_clear_error();

typedef void (*KFn)(McVol);         // per-volume kernel: one volume by value
typedef void (*KFnB)(McBatchSrc);   // batched twin: many volumes of one class

struct KPair {
    KFn plain;
    KFnB batch;
    int threads;   // work-group size of both
};

KPair mc_pick_range_u8();
KPair mc_pick_range_u16();
KPair mc_pick_range_f32();
KPair mc_pick_hist_u8(bool ahr, bool ro, int peel);
KPair mc_pick_hist_u16(bool ahr, bool ro, int peel);
KPair mc_pick_hist_f32(bool ahr, bool ro, int peel);
KPair mc_pick_map_u8(int D, bool ahr, int path);
KPair mc_pick_map_u16(int D, bool ahr, int path);
KPair mc_pick_map_f32(int D, bool ahr, int path);
