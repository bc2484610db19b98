// Internal interface between the host runtime and the kernel translation
// units of the MCLAHE library.
#pragma once
#include "mc_desc.h"

typedef void (*KFn)(McVol);

KFn mc_pick_range_u8();
KFn mc_pick_range_u16();
KFn mc_pick_range_f32();
KFn mc_pick_hist_u8(bool ahr, bool ro, int peel);
KFn mc_pick_hist_u16(bool ahr, bool ro, int peel);
KFn mc_pick_hist_f32(bool ahr, bool ro, int peel);
KFn mc_pick_map_u8(int D, bool ahr, int path);
KFn mc_pick_map_u16(int D, bool ahr, int path);
KFn mc_pick_map_f32(int D, bool ahr, int path);

// Persistent batched kernel (k_persist.hip): host-side kernel handles.
const void *mc_persistent_fn();
const void *mc_zero_fn();
