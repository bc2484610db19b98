// Per-volume and batched kernels instantiated for float input.
#include "mc_plain_kernels.h"

KPair mc_pick_range_f32() { return KPair{(KFn)k_range_ghr<float>, (KFnB)k_range_ghr_b<float>, MC_T}; }
KPair mc_pick_hist_f32(bool ahr, bool ro, int peel) { return pick_hist_t<float>(ahr, ro, peel); }
KPair mc_pick_map_f32(int D, bool ahr, int path) { return pick_map_t2<float>(D, ahr, path); }
KFn mc_pick_map_met_f32(int D, bool ahr, int path) { return pick_map_met_t2<float>(D, ahr, path); }
