// Per-volume and batched kernels instantiated for uint16_t input.
#include "mc_plain_kernels.h"

KPair mc_pick_range_u16() { return KPair{(KFn)k_range_ghr<uint16_t>, (KFnB)k_range_ghr_b<uint16_t>, MC_T}; }
KPair mc_pick_hist_u16(bool ahr, bool ro, int peel) { return pick_hist_t<uint16_t>(ahr, ro, peel); }
KPair mc_pick_map_u16(int D, bool ahr, int path) { return pick_map_t2<uint16_t>(D, ahr, path); }
KFn mc_pick_map_met_u16(int D, bool ahr, int path) { return pick_map_met_t2<uint16_t>(D, ahr, path); }
