// Host-only probe of the library's shared geometry helpers (mc_desc.h), so
// that the virtual-padding footprints and interpolation cells can be checked
// on the CPU against numpy's symmetric padding.
#include "mc_desc.h"

extern "C" {
// box of kernel k: out[0..3] = lo, hi, olo, ohi
void probe_kernel_box(int s, int b, int p0, int p1, int k, int *out)
{
    McAxis a{s, b, p0, p1, (s + p0 + p1) / b};
    McBox r = mc_kernel_box(a, k);
    out[0] = r.lo;
    out[1] = r.hi;
    out[2] = r.olo;
    out[3] = r.ohi;
}
void probe_cell_range(int s, int b, int p0, int p1, int c, int *out)
{
    McAxis a{s, b, p0, p1, (s + p0 + p1) / b};
    mc_cell_range(a, c, out[0], out[1]);
    out[2] = out[0] < out[1] ? mc_cell_m(a, c, out[0]) : -1;
}
}
