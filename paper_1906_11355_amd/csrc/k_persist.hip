// The persistent batched kernel: one launch runs every work unit of every
// pass of every volume of a batch, taking tickets in order from one counter
// (the protocol and why it cannot deadlock: mc_persist.h).  Each unit runs
// the same unit function as the per-pass kernels, so the outputs are
// bit-identical to theirs; interpolation units run with MC_T threads here
// (per voxel the arithmetic does not depend on the thread mapping).
#include "mc_kernels.h"
#include "mc_launch.h"
#include "mc_persist.h"

namespace {

// Device side of the protocol's atomics.  A peek is an agent-scope atomic
// load (it may be served by the local L2, so it may see an older value).  A
// poll is an atomic
// read-modify-write at agent scope, performed where the updates of every
// XCD meet whatever the local L2 holds: a compare-and-swap against a value
// no run word ever takes, so it never stores and returns the current value
// (an idempotent fetch-or or fetch-add would be turned into a plain load).
// The abort word is set once, by compare-and-swap from zero.
struct DevAtomics {
    static __device__ __forceinline__ uint32_t peek(uint32_t *p)
    {
        return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ uint32_t poll(uint32_t *p)
    {
        uint32_t v = 0xffffffffu;
        __hip_atomic_compare_exchange_strong(p, &v, 0xffffffffu, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
        return v;
    }
    static __device__ __forceinline__ void set_abort(uint32_t *p, uint32_t v)
    {
        uint32_t z = 0;
        __hip_atomic_compare_exchange_strong(p, &z, v, __ATOMIC_RELAXED, __ATOMIC_RELAXED,
                                             __HIP_MEMORY_SCOPE_AGENT);
    }
    static __device__ __forceinline__ void sleep() { __builtin_amdgcn_s_sleep(8); }
};

// Each kind of unit is its own (not inlined) function, so that the kernel
// needs the registers of the heaviest one, not of all of them at once.
template <typename Tin, bool AHR, bool RO, bool VAL = false>
__device__ __noinline__ void pu_hist(const McVol &v, uint32_t u, char *smem)
{
    // wavefront aggregation changes no count: the plain update serves all
    mc::hist_unit_dispatch<Tin, AHR, RO, 0, VAL, 2>(v, u, smem);
}
template <typename Tin>
__device__ __noinline__ void pu_range(const McVol &v, uint32_t u, char *smem)
{
    mc::range_ghr_unit<Tin>(v, u, smem);
}
__device__ __noinline__ void pu_clip(const McVol &v, uint32_t u, char *smem) { mc::clip_unit(v, u, smem); }
template <typename Tin, int D, bool AHR>
__device__ __noinline__ void pu_map(const McVol &v, uint32_t u, char *smem)
{
    mc::map_unit<Tin, D, AHR, false, MC_T>(v, u, smem);
}
template <typename Tin, bool AHR>
__device__ __noinline__ void pu_map_generic(const McVol &v, uint32_t u, char *smem)
{
    mc::map_unit_generic<Tin, AHR>(v, u, smem);
}

template <typename Tin>
__device__ void persist_unit(const McVol &v, uint32_t ph, uint32_t u, char *smem)
{
    const bool ahr = v.mode == MC_AHR;
    if (ph == 0) {
        if (ahr) pu_hist<Tin, true, true>(v, u, smem);
        else pu_range<Tin>(v, u, smem);
    } else if (ph == 1) {
        if constexpr (sizeof(Tin) == 1) {
            if (v.vhist) {   // uint8 counted per value
                if (ahr) pu_hist<Tin, true, false, true>(v, u, smem);
                else pu_hist<Tin, false, false, true>(v, u, smem);
                return;
            }
        }
        if (ahr) pu_hist<Tin, true, false>(v, u, smem);
        else pu_hist<Tin, false, false>(v, u, smem);
    } else if (ph == 2) {
        pu_clip(v, u, smem);
    } else if (v.path) {
        if (ahr) pu_map_generic<Tin, true>(v, u, smem);
        else pu_map_generic<Tin, false>(v, u, smem);
    } else if (ahr) {
        switch (v.D) {
        case 1: pu_map<Tin, 1, true>(v, u, smem); break;
        case 2: pu_map<Tin, 2, true>(v, u, smem); break;
        case 3: pu_map<Tin, 3, true>(v, u, smem); break;
        default: pu_map<Tin, 4, true>(v, u, smem); break;
        }
    } else {
        switch (v.D) {
        case 1: pu_map<Tin, 1, false>(v, u, smem); break;
        case 2: pu_map<Tin, 2, false>(v, u, smem); break;
        case 3: pu_map<Tin, 3, false>(v, u, smem); break;
        default: pu_map<Tin, 4, false>(v, u, smem); break;
        }
    }
}

// Two waves per SIMD (up to 256 VGPRs): every kind of unit then runs
// without spilling (at three or four waves the called unit functions spill
// to scratch inside their loops); each unit keeps many loads in flight.
//
// Control flow is kept uniform across the work-group on purpose: the ticket
// and its decoding are read back with readfirstlane (scalar values), so the
// loop exit and the unit dispatch are scalar branches, and thread 0's work
// is one guarded block per iteration (it first signals the previous ticket's
// completion, then takes the next ticket).  A loop whose exit depends on
// values the compiler takes for per-lane ones, with thread 0 guarded both at
// the end of an iteration and at the start of the next, was compiled into
// two nested loops: the other lanes went back to the barrier without the
// outer loop in which thread 0 takes tickets, so a work-group re-ran its
// unit forever and the launch never ended.
// vols: the descriptors again, as a restrict parameter (read with scalar
// loads; the table is not written during the launch)
__global__ __launch_bounds__(MC_T, 2) void k_persist(McPersistSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    __shared__ uint32_t info[4];
    const McPersistHdr &h = *s.hdr;
    const uint32_t total = h.total;
    uint32_t *prev = nullptr;   // thread 0: counter of the ticket it ran last
    uint32_t prev_ph = MC_PHASES;   // pass of the previous ticket (uniform)
    for (;;) {
        // every thread's writes of the previous unit, visible device-wide
        // before its counter moves.  Interpolation output is read by no
        // later unit: no release after an interpolation unit.
        if (prev_ph < MC_PHASES - 1) __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        __syncthreads();
        if (threadIdx.x == 0) {
            if (prev) __hip_atomic_fetch_add(prev, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint32_t t = __hip_atomic_fetch_add(&s.q[MC_PQ_HEAD], 1u, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT);
            McTicket k = {0u, 0u, 0u};
            uint32_t go = 0;
            if (t < total) {
                k = mc_ticket(h, s.pre, t);
                go = mc_persist_wait<DevAtomics>(h, s.pre, s.q, k, t) ? 1u : 0u;
                // only a unit that ran counts: after an abort, the units of
                // a skipped unit's volume wait and see the abort word instead
                // of running on what the skipped one did not write
                prev = go ? mc_persist_done(h, s.q, k) : nullptr;
            } else {
                prev = nullptr;
            }
            info[0] = t;
            info[1] = k.phase;
            info[2] = k.vol;
            info[3] = k.unit | (go << 31);
        }
        __syncthreads();
        const uint32_t t = __builtin_amdgcn_readfirstlane(info[0]);
        const uint32_t ph = __builtin_amdgcn_readfirstlane(info[1]);
        const uint32_t vi = __builtin_amdgcn_readfirstlane(info[2]);
        const uint32_t uw = __builtin_amdgcn_readfirstlane(info[3]);
        if (t >= total) break;
        prev_ph = ph;
        if (uw >> 31) {
            // the producers' writes (released before their counters moved);
            // the range pass reads only the input
            if (ph > 0) __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const McVol &v = vols[vi];
            mc::warm_desc(v);
            const uint32_t u = uw & 0x7fffffffu;
            if (v.in_dt == MC_U8) persist_unit<uint8_t>(v, ph, u, smem);
            else if (v.in_dt == MC_U16) persist_unit<uint16_t>(v, ph, u, smem);
            else persist_unit<float>(v, ph, u, smem);
        }
    }
}

// Clears the run's words before the persistent launch (a kernel, so that a
// captured graph holds no memset node).
__global__ __launch_bounds__(MC_T) void k_persist_reset(uint32_t *q, uint32_t n)
{
    for (uint32_t i = blockIdx.x * MC_T + threadIdx.x; i < n; i += gridDim.x * MC_T) q[i] = 0u;
}

}  // namespace

const void *mc_persist_fn() { return (const void *)k_persist; }
const void *mc_persist_reset_fn() { return (const void *)k_persist_reset; }
