// Per-pass kernels of the plain (one volume per call) path, as templates.
// Each k_plain_<dtype>.hip instantiates them for one input dtype so that the
// translation units compile in parallel.
#pragma once
#include "mc_kernels.h"
#include "mc_launch.h"

// Every kernel has a batched twin (suffix _b) that serves one pass of many
// volumes of the same class: it finds its volume and unit in the launch's
// index table and runs the very same unit function.  The volume descriptors
// come as a kernel parameter of their own, declared restrict (the table is
// written before the launch and only read during it): the compiler then
// reads the descriptor with scalar loads and keeps its fields, as for a
// descriptor passed by value, instead of reloading them with vector loads
// after every store that might have written the table.
__device__ __forceinline__ const McVol &mc_resolve(const McBatchSrc &s, const McVol *__restrict__ vols,
                                                   uint32_t &u)
{
    // the volume and unit are the work-group's own: scalar values
    const uint32_t r = blockIdx.x;
    const uint32_t j = __builtin_amdgcn_readfirstlane(mc_batch_volume(s.pre, s.n, r));
    u = __builtin_amdgcn_readfirstlane(r - s.pre[j]);
    const uint32_t vi = __builtin_amdgcn_readfirstlane(s.list[j]);
    mc::warm_desc(vols[vi]);
    return vols[vi];
}

template <typename Tin>
__global__ __launch_bounds__(MC_T) void k_range_ghr(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::range_ghr_unit<Tin>(d, blockIdx.x, smem);
}
template <typename Tin>
__global__ __launch_bounds__(MC_T) void k_range_ghr_b(McBatchSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t u;
    const McVol &d = mc_resolve(s, vols, u);
    mc::range_ghr_unit<Tin>(d, u, smem);
}

template <typename Tin, bool AHR, bool RO, int PEEL, bool VAL = false>
__global__ __launch_bounds__(MC_T) void k_hist(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    // wave aggregation needs the registers of two rows per step (four spill)
    mc::hist_unit_dispatch<Tin, AHR, RO, PEEL, VAL, (PEEL > 0 ? 2 : 4)>(d, blockIdx.x, smem);
}
template <typename Tin, bool AHR, bool RO, int PEEL, bool VAL = false>
__global__ __launch_bounds__(MC_T) void k_hist_b(McBatchSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t u;
    const McVol &d = mc_resolve(s, vols, u);
    mc::hist_unit_dispatch<Tin, AHR, RO, PEEL, VAL, 2>(d, u, smem);
}

template <typename Tin, int D, bool AHR>
__global__ __launch_bounds__(mc_map_threads(AHR), 4) void k_map(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::map_unit<Tin, D, AHR>(d, blockIdx.x, smem);
}
template <typename Tin, int D, bool AHR>
__global__ __launch_bounds__(mc_map_threads(AHR), 4) void k_map_b(McBatchSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t u;
    const McVol &d = mc_resolve(s, vols, u);
    mc::map_unit<Tin, D, AHR>(d, u, smem);
}

template <typename Tin, bool AHR>
__global__ __launch_bounds__(MC_T) void k_map_generic(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::map_unit_generic<Tin, AHR>(d, blockIdx.x, smem);
}
template <typename Tin, bool AHR>
__global__ __launch_bounds__(MC_T) void k_map_generic_b(McBatchSrc s, const McVol *__restrict__ vols)
{
    extern __shared__ __align__(16) char smem[];
    uint32_t u;
    const McVol &d = mc_resolve(s, vols, u);
    mc::map_unit_generic<Tin, AHR>(d, u, smem);
}

// Interpolation with the contrast-metric epilogue (per-volume runs only):
// the same unit function, which also writes each unit's input and output
// statistics.
template <typename Tin, int D, bool AHR>
__global__ __launch_bounds__(mc_map_threads(AHR), 4) void k_map_m(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::map_unit<Tin, D, AHR, true>(d, blockIdx.x, smem);
}
template <typename Tin, bool AHR>
__global__ __launch_bounds__(MC_T) void k_map_generic_m(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::warm_desc(d);
    mc::map_unit_generic<Tin, AHR, true>(d, blockIdx.x, smem);
}

template <typename Tin, bool AHR>
static KFn pick_map_met_t(int D, int path)
{
    if (path) return (KFn)k_map_generic_m<Tin, AHR>;
    switch (D) {
    case 1: return (KFn)k_map_m<Tin, 1, AHR>;
    case 2: return (KFn)k_map_m<Tin, 2, AHR>;
    case 3: return (KFn)k_map_m<Tin, 3, AHR>;
    default: return (KFn)k_map_m<Tin, 4, AHR>;
    }
}

template <typename Tin>
static KFn pick_map_met_t2(int D, bool ahr, int path)
{
    return ahr ? pick_map_met_t<Tin, true>(D, path) : pick_map_met_t<Tin, false>(D, path);
}

template <typename Tin, bool AHR, bool RO, int PEEL, bool VAL = false>
static KPair hist_pair()
{
    return KPair{(KFn)k_hist<Tin, AHR, RO, PEEL, VAL>, (KFnB)k_hist_b<Tin, AHR, RO, PEEL, VAL>, MC_T};
}

template <typename Tin>
static KPair pick_hist_t(bool ahr, bool ro, int peel, bool val = false)
{
    if constexpr (sizeof(Tin) == 1) {
        if (val && !ro) {
            if (ahr) return peel == 0 ? hist_pair<Tin, true, false, 0, true>() : hist_pair<Tin, true, false, 1, true>();
            return peel == 0 ? hist_pair<Tin, false, false, 0, true>() : hist_pair<Tin, false, false, 1, true>();
        }
    }
    if (ro) return hist_pair<Tin, true, true, 0>();
    if (ahr) return peel == 0 ? hist_pair<Tin, true, false, 0>() : hist_pair<Tin, true, false, 1>();
    return peel == 0 ? hist_pair<Tin, false, false, 0>() : hist_pair<Tin, false, false, 1>();
}

template <typename Tin, int D, bool AHR>
static KPair map_pair() { return KPair{(KFn)k_map<Tin, D, AHR>, (KFnB)k_map_b<Tin, D, AHR>, mc_map_threads(AHR)}; }

template <typename Tin, bool AHR>
static KPair pick_map_t(int D, int path)
{
    if (path) return KPair{(KFn)k_map_generic<Tin, AHR>, (KFnB)k_map_generic_b<Tin, AHR>, MC_T};
    switch (D) {
    case 1: return map_pair<Tin, 1, AHR>();
    case 2: return map_pair<Tin, 2, AHR>();
    case 3: return map_pair<Tin, 3, AHR>();
    default: return map_pair<Tin, 4, AHR>();
    }
}

template <typename Tin>
static KPair pick_map_t2(int D, bool ahr, int path)
{
    return ahr ? pick_map_t<Tin, true>(D, path) : pick_map_t<Tin, false>(D, path);
}
