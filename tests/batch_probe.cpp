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
}
