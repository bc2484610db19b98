// Host-only probe of the batched descriptor table: decodes every work-group
// of every batched launch with the same functions the batched kernels use
// (mc_batch_volume, mc_phase_units) and checks that each unit of each pass of
// each volume is visited exactly once.
#include <stdint.h>
#include <string.h>

#include <vector>

#include "mc_desc.h"

static uint64_t a256(uint64_t x) { return (x + 255) & ~uint64_t(255); }

extern "C" {
// counts[ph * nvol + v] = units of pass ph decoded to volume v; ptrs[v*3..] =
// in, out and hist pointers of volume v; *nlaunch = launches of the batch.
// Returns 0 if every unit of every volume is decoded exactly once.
int probe_batch(const char *img, size_t size, uint32_t *counts, uint64_t *ptrs, uint32_t *nlaunch)
{
    const McBatchHdr *h = (const McBatchHdr *)img;
    const uint32_t n = h->nvol;
    const uint64_t o_recs = a256(sizeof(McBatchHdr));
    const McLaunchRec *recs = (const McLaunchRec *)(img + o_recs);
    const uint64_t o_idx = a256(o_recs + (uint64_t)h->nlaunch * sizeof(McLaunchRec));
    const uint32_t *idx = (const uint32_t *)(img + o_idx);
    uint64_t n_idx = 0;
    for (uint32_t j = 0; j < h->nlaunch; ++j) n_idx += 2 * (uint64_t)recs[j].n + 1;
    const uint64_t o_vols = a256(o_idx + n_idx * 4);
    if (o_vols + (uint64_t)n * sizeof(McVol) > size) return 1;
    const McVol *vols = (const McVol *)(img + o_vols);
    std::vector<std::vector<std::vector<uint8_t>>> seen(MC_PHASES, std::vector<std::vector<uint8_t>>(n));
    for (int ph = 0; ph < MC_PHASES; ++ph)
        for (uint32_t v = 0; v < n; ++v) seen[ph][v].assign(mc_phase_units(vols[v], ph), 0);
    int last_phase = -1;
    for (uint32_t j = 0; j < h->nlaunch; ++j) {
        const McLaunchRec &r = recs[j];
        if ((int)r.phase < last_phase || r.phase >= MC_PHASES) return 2;   // passes in order
        last_phase = (int)r.phase;
        const uint32_t *list = idx + r.list, *pre = idx + r.pre;
        if (pre[0] != 0 || pre[r.n] != r.units) return 3;
        for (uint32_t g = 0; g < r.units; ++g) {
            const uint32_t e = mc_batch_volume(pre, r.n, g);
            if (e >= r.n) return 4;
            const uint32_t v = list[e], u = g - pre[e];
            if (v >= n || u >= seen[r.phase][v].size()) return 5;
            if (seen[r.phase][v][u]++) return 6;
        }
    }
    for (int ph = 0; ph < MC_PHASES; ++ph)
        for (uint32_t v = 0; v < n; ++v) {
            for (uint8_t c : seen[ph][v])
                if (c != 1) return 7;
            counts[ph * n + v] = (uint32_t)seen[ph][v].size();
        }
    for (uint32_t v = 0; v < n; ++v) {
        ptrs[3 * v] = (uint64_t)(uintptr_t)vols[v].in;
        ptrs[3 * v + 1] = (uint64_t)(uintptr_t)vols[v].out;
        ptrs[3 * v + 2] = (uint64_t)(uintptr_t)vols[v].hist;
    }
    *nlaunch = h->nlaunch;
    return 0;
}

// Largest number of load chunks (V elements each) in one row segment of a
// histogram unit and of an interpolation unit of every volume of the table,
// restating how the units cut the last axis: histogram segments of hG kernel
// footprints (or part pp of hP parts of one footprint), interpolation groups
// of mG cells (or part pp of mP parts of one cell).  A unit's threads cover a
// segment only if it has at most as many chunks as the work-group has
// threads.  Returns 0 and fills hist_max / map_max per volume.
int probe_batch_chunks(const char *img, size_t size, uint32_t *hist_max, uint32_t *map_max, uint32_t *vec)
{
    const McBatchHdr *h = (const McBatchHdr *)img;
    const uint32_t n = h->nvol;
    const uint64_t o_recs = a256(sizeof(McBatchHdr));
    const McLaunchRec *recs = (const McLaunchRec *)(img + o_recs);
    const uint64_t o_idx = a256(o_recs + (uint64_t)h->nlaunch * sizeof(McLaunchRec));
    uint64_t n_idx = 0;
    for (uint32_t j = 0; j < h->nlaunch; ++j) n_idx += 2 * (uint64_t)recs[j].n + 1;
    const uint64_t o_vols = a256(o_idx + n_idx * 4);
    if (o_vols + (uint64_t)n * sizeof(McVol) > size) return 1;
    const McVol *vols = (const McVol *)(img + o_vols);
    for (uint32_t i = 0; i < n; ++i) {
        const McVol &v = vols[i];
        const McAxis &a = v.ax[v.D - 1];
        const int V = v.vec;
        auto chunks = [V](int xs, int xe) { return xe > xs ? (xe + V - 1) / V - xs / V : 0; };
        int hm = 0;
        for (int j = 0; j < v.hS; ++j) {
            int xs = 0x7fffffff, xe = -1;
            if (v.hP == 1) {
                for (int k = j * v.hG; k < mc_min((j + 1) * v.hG, a.n); ++k) {
                    const McBox b = mc_kernel_box(a, k);
                    xs = mc_min(xs, b.lo);
                    xe = mc_max(xe, b.hi);
                }
            } else {
                const McBox b = mc_kernel_box(a, j / v.hP);
                const int pp = j % v.hP, len = b.hi - b.lo;
                xs = b.lo + (int)((int64_t)len * pp / v.hP);
                xe = b.lo + (int)((int64_t)len * (pp + 1) / v.hP);
            }
            hm = mc_max(hm, chunks(xs, xe));
        }
        int mm = 0;
        if (v.path == 0) {
            for (int g = 0; g < v.mS; ++g) {
                int xs, xe, t;
                if (v.mP == 1) {
                    mc_cell_range(a, g * v.mG, xs, t);
                    mc_cell_range(a, mc_min((g + 1) * v.mG, a.n - 1) - 1, t, xe);
                } else {
                    int lo, hi;
                    mc_cell_range(a, g / v.mP, lo, hi);
                    const int pp = g % v.mP;
                    xs = lo + (int)((int64_t)(hi - lo) * pp / v.mP);
                    xe = lo + (int)((int64_t)(hi - lo) * (pp + 1) / v.mP);
                }
                mm = mc_max(mm, chunks(xs, xe));
            }
        }
        hist_max[i] = (uint32_t)hm;
        map_max[i] = (uint32_t)mm;
        vec[i] = (uint32_t)V;
    }
    return 0;
}
}
