// Per-volume and batched kernels instantiated for uint8_t input.
#include "mc_plain_kernels.h"

KPair mc_pick_range_u8() { return KPair{(KFn)k_range_ghr<uint8_t>, (KFnB)k_range_ghr_b<uint8_t>, MC_T}; }
KPair mc_pick_hist_u8(bool ahr, bool ro, int peel, bool val) { return pick_hist_t<uint8_t>(ahr, ro, peel, val); }
KPair mc_pick_map_u8(int D, bool ahr, int path) { return pick_map_t2<uint8_t>(D, ahr, path); }
KFn mc_pick_map_met_u8(int D, bool ahr, int path) { return pick_map_met_t2<uint8_t>(D, ahr, path); }
