// Plain-path kernels instantiated for uint8_t input.
#include "mc_plain_kernels.h"

KFn mc_pick_range_u8() { return (KFn)k_range_ghr<uint8_t>; }
KFn mc_pick_hist_u8(bool ahr, bool ro, int peel) { return pick_hist_t<uint8_t>(ahr, ro, peel); }
KFn mc_pick_map_u8(int D, bool ahr, int path) { return pick_map_t2<uint8_t>(D, ahr, path); }
