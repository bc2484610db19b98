// Per-pass kernels of the plain (one volume per call) path, as templates.
// Each k_plain_<dtype>.hip instantiates them for one input dtype so that the
// translation units compile in parallel.
#pragma once
#include "mc_kernels.h"
#include "mc_launch.h"

template <typename Tin>
__global__ __launch_bounds__(MC_T) void k_range_ghr(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::range_ghr_unit<Tin>(d, blockIdx.x, smem);
}

template <typename Tin, bool AHR, bool RO, int PEEL>
__global__ __launch_bounds__(MC_T) void k_hist(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::hist_unit_dispatch<Tin, AHR, RO, PEEL>(d, blockIdx.x, smem);
}

template <typename Tin, int D, bool AHR>
__global__ __launch_bounds__(MC_T) void k_map(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::map_unit<Tin, D, AHR>(d, blockIdx.x, smem);
}

template <typename Tin, bool AHR>
__global__ __launch_bounds__(MC_T) void k_map_generic(McVol d)
{
    extern __shared__ __align__(16) char smem[];
    mc::map_unit_generic<Tin, AHR>(d, blockIdx.x, smem);
}


template <typename Tin>
static KFn pick_hist_t(bool ahr, bool ro, int peel)
{
    if (ro) return (KFn)k_hist<Tin, true, true, 0>;
    if (ahr) return peel == 0 ? (KFn)k_hist<Tin, true, false, 0>
                  : peel == 1 ? (KFn)k_hist<Tin, true, false, 1> : (KFn)k_hist<Tin, true, false, 2>;
    return peel == 0 ? (KFn)k_hist<Tin, false, false, 0>
         : peel == 1 ? (KFn)k_hist<Tin, false, false, 1> : (KFn)k_hist<Tin, false, false, 2>;
}

template <typename Tin, bool AHR>
static KFn pick_map_t(int D, int path)
{
    if (path) return (KFn)k_map_generic<Tin, AHR>;
    switch (D) {
    case 1: return (KFn)k_map<Tin, 1, AHR>;
    case 2: return (KFn)k_map<Tin, 2, AHR>;
    case 3: return (KFn)k_map<Tin, 3, AHR>;
    default: return (KFn)k_map<Tin, 4, AHR>;
    }
}

template <typename Tin>
static KFn pick_map_t2(int D, bool ahr, int path)
{
    return ahr ? pick_map_t<Tin, true>(D, path) : pick_map_t<Tin, false>(D, path);
}

