// LDS atomic-add throughput probe for gfx950 (measurement tooling; not part
// of the MCLAHE library or its ABI).
//
// Every thread issues `iters` 32-bit LDS atomic adds (ds_add_u32, no return).
// The 64 lanes of a wave spread over `ways` distinct addresses: ways = 64 is
// conflict-free (consecutive words), ways = 1 sends the whole wave to one
// word, values in between share each word among 64/ways lanes.  The address
// set rotates over 8 disjoint blocks from one iteration to the next, so no
// two consecutive atomics of a lane touch the same word.  All addresses lie
// in a 64*8*4 = 2 KiB array per wave.
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PROBE_T 256
#define PROBE_WAVES (PROBE_T / 64)

__global__ __launch_bounds__(PROBE_T) void k_lds_atomics(uint32_t *out, int iters, int ways)
{
    __shared__ uint32_t h[PROBE_WAVES][8][64];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < PROBE_WAVES * 8 * 64; i += PROBE_T) (&h[0][0][0])[i] = 0;
    __syncthreads();
    const int slot = lane % ways;      // 0 <= slot < ways <= 64
    for (int i = 0; i < iters; ++i) atomicAdd(&h[wave][i & 7][slot], 1u);
    __syncthreads();
    uint32_t s = 0;
    for (int b = 0; b < 8; ++b) s += h[wave][b][lane];
    // one value per thread keeps the adds live; the host checks the total
    atomicAdd(out, s);
}

extern "C" {

// Launch `blocks` work-groups of 256 threads on `stream`, time them with HIP
// events and synchronise.  *ms = kernel time, *lane_ops = atomics issued.
// Returns 0, or -1 for bad arguments, or the HIP error code.  d_out must be a
// zeroed device uint32; after the call it holds blocks * 256 * iters.
int mclahe_probe_lds_atomics(int ways, int iters, int blocks, uint32_t *d_out, void *stream, float *ms,
                             unsigned long long *lane_ops)
{
    if (ways < 1 || ways > 64 || (64 % ways) || iters < 1 || blocks < 1 || !d_out || !ms || !lane_ops) return -1;
    hipStream_t st = (hipStream_t)stream;
    hipEvent_t a, b;
    hipError_t e;
    if ((e = hipEventCreate(&a)) != hipSuccess) return (int)e;
    if ((e = hipEventCreate(&b)) != hipSuccess) {
        (void)hipEventDestroy(a);
        return (int)e;
    }
    (void)hipEventRecord(a, st);
    hipLaunchKernelGGL(k_lds_atomics, dim3(blocks), dim3(PROBE_T), 0, st, d_out, iters, ways);
    e = hipGetLastError();
    (void)hipEventRecord(b, st);
    if (e == hipSuccess) e = hipEventSynchronize(b);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, a, b);
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    *lane_ops = (unsigned long long)blocks * PROBE_T * (unsigned long long)iters;
    return (int)e;
}

}
