// Plain-path kernels instantiated for uint16_t input.
#include "mc_plain_kernels.h"

KFn mc_pick_range_u16() { return (KFn)k_range_ghr<uint16_t>; }
KFn mc_pick_hist_u16(bool ahr, bool ro, int peel) { return pick_hist_t<uint16_t>(ahr, ro, peel); }
KFn mc_pick_map_u16(int D, bool ahr, int path) { return pick_map_t2<uint16_t>(D, ahr, path); }
