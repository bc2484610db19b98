// Persistent batched kernel of the MCLAHE library: one launch runs every
// unit of every volume of a batch, pulled from a phase-ordered ticket queue.
#include "mc_kernels.h"
#include "mc_launch.h"

__device__ __forceinline__ uint32_t phase_units(const McVol &v, int ph)
{
    switch (ph) {
    case 0: return v.mode == MC_AHR ? v.n_hist_wu : v.n_range_wu;
    case 1: return v.n_hist_wu;
    case 2: return v.n_clip_wu;
    default: return v.n_map_wu;
    }
}

template <typename Tin>
__device__ void unit_dispatch(const McVol &v, int ph, uint32_t u, char *smem)
{
    const bool ahr = v.mode == MC_AHR;
    if (ph == 0) {
        if (ahr) mc::hist_unit_dispatch<Tin, true, true, 0>(v, u, smem);
        else mc::range_ghr_unit<Tin>(v, u, smem);
    } else if (ph == 1) {
        if (ahr) {
            if (v.hPeel == 0) mc::hist_unit_dispatch<Tin, true, false, 0>(v, u, smem);
            else if (v.hPeel == 1) mc::hist_unit_dispatch<Tin, true, false, 1>(v, u, smem);
            else mc::hist_unit_dispatch<Tin, true, false, 2>(v, u, smem);
        } else {
            if (v.hPeel == 0) mc::hist_unit_dispatch<Tin, false, false, 0>(v, u, smem);
            else if (v.hPeel == 1) mc::hist_unit_dispatch<Tin, false, false, 1>(v, u, smem);
            else mc::hist_unit_dispatch<Tin, false, false, 2>(v, u, smem);
        }
    } else if (ph == 2) {
        mc::clip_unit(v, u, smem);
    } else {
        if (v.path) {
            if (ahr) mc::map_unit_generic<Tin, true>(v, u, smem);
            else mc::map_unit_generic<Tin, false>(v, u, smem);
        } else if (ahr) {
            switch (v.D) {
            case 1: mc::map_unit<Tin, 1, true>(v, u, smem); break;
            case 2: mc::map_unit<Tin, 2, true>(v, u, smem); break;
            case 3: mc::map_unit<Tin, 3, true>(v, u, smem); break;
            default: mc::map_unit<Tin, 4, true>(v, u, smem); break;
            }
        } else {
            switch (v.D) {
            case 1: mc::map_unit<Tin, 1, false>(v, u, smem); break;
            case 2: mc::map_unit<Tin, 2, false>(v, u, smem); break;
            case 3: mc::map_unit<Tin, 3, false>(v, u, smem); break;
            default: mc::map_unit<Tin, 4, false>(v, u, smem); break;
            }
        }
    }
}

// Work-queue kernel.  A work-group takes the next ticket, waits until the
// phase its unit depends on is complete for that volume, runs the unit and
// publishes its completion.  Tickets are issued in dependency order (phase
// major), so every unit a waiter depends on was taken earlier by a running
// work-group: the queue cannot deadlock, and each wait is bounded anyway.
__global__ __launch_bounds__(MC_T) void k_persistent(const McBatch *hdr, const uint32_t *vstart,
                                                     const McVol *vols, McQueue *q,
                                                     uint32_t *done)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t s_info[4];
    const uint32_t nvol = hdr->nvol, total = hdr->total;
    for (;;) {
        if (threadIdx.x == 0) {
            const uint32_t t = __hip_atomic_fetch_add(&q->head, 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            uint32_t ph = 0, vi = 0, u = 0, ok = 1;
            if (t < total) {
                while (ph + 1 < MC_PHASES && t >= hdr->phase_start[ph + 1]) ++ph;
                const uint32_t r = t - hdr->phase_start[ph];
                const uint32_t *vs = vstart + ph * (nvol + 1);
                uint32_t lo = 0, hi = nvol;   // largest vi with vs[vi] <= r
                while (hi - lo > 1) {
                    const uint32_t mid = (lo + hi) / 2;
                    if (vs[mid] <= r) lo = mid;
                    else hi = mid;
                }
                vi = lo;
                u = r - vs[vi];
                if (ph > 0) {
                    const uint32_t need = phase_units(vols[vi], ph - 1);
                    uint32_t *cnt = done + (ph - 1) * nvol + vi;
                    uint32_t spins = 0;
                    while (__hip_atomic_load(cnt, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < need) {
                        __builtin_amdgcn_s_sleep(2);
                        if (++spins > hdr->spin_limit) {
                            __hip_atomic_store(&q->error, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                            ok = 0;
                            break;
                        }
                    }
                }
            }
            s_info[0] = t;
            s_info[1] = ph;
            s_info[2] = vi;
            s_info[3] = (u & 0x7fffffffu) | (ok ? 0u : 0x80000000u);
        }
        __syncthreads();
        const uint32_t t = s_info[0], ph = s_info[1], vi = s_info[2], ui = s_info[3];
        __syncthreads();
        if (t >= total) break;
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        const McVol &v = vols[vi];
        if (!(ui & 0x80000000u)) {
            const uint32_t u = ui & 0x7fffffffu;
            if (v.in_dt == MC_U8) unit_dispatch<uint8_t>(v, (int)ph, u, smem);
            else if (v.in_dt == MC_U16) unit_dispatch<uint16_t>(v, (int)ph, u, smem);
            else unit_dispatch<float>(v, (int)ph, u, smem);
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0)
            __hip_atomic_fetch_add(done + ph * nvol + vi, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
}

// Reset of the queue header and the completion counters (a plain kernel, so
// that the graph holds no memset node).
__global__ void k_zero_words(uint32_t *p, uint32_t n)
{
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n; i += gridDim.x * blockDim.x) p[i] = 0;
}


const void *mc_persistent_fn() { return (const void *)k_persistent; }
const void *mc_zero_fn() { return (const void *)k_zero_words; }
