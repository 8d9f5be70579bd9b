// Persistent launches of the MacLABSWE step: many passes in one launch
// (cooperative grid barrier between passes).
#include "mlb_step_impl.h"

namespace mlb {

// Many passes in one cooperative launch, every tile's wave resident: a grid
// barrier on a device counter separates the passes, so small grids do not
// pay a launch per pass.  Every workgroup arrives once per pass (idle waves
// included).  Waiting is bounded: after spin_limit polls, or once another
// workgroup has given up, the error flag is set and every workgroup leaves
// the loop at that barrier, so the grid always drains.
template <int KIND, bool MASKED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(2)))
void persistent_kernel(const BasinDev* __restrict__ basins, const TileDev* __restrict__ tiles, int ntiles,
                       int parity0, int npasses, SyncState* __restrict__ sync, uint64_t base, int spin_limit)
{
    __shared__ int abort_flag;
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    const uint64_t nblk = gridDim.x;
    // an earlier launch gave up: do nothing until the host has reset the state
    if (threadIdx.x == 0) abort_flag = __hip_atomic_load(&sync->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    if (abort_flag) return;
    for (int p = 0; p < npasses; ++p) {
        if (t < ntiles)
            pass_tile<KIND, false, MASKED, false, false, false>(basins, tiles, t, parity0 ^ (p & 1), nullptr,
                                                                CoherentStep{});
        __threadfence();   // release: this wave's stores, device-wide
        __syncthreads();
        if (threadIdx.x == 0) {
            __hip_atomic_fetch_add(&sync->count, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t target = base + (uint64_t)(p + 1) * nblk;
            int spins = 0;
            while (__hip_atomic_load(&sync->count, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < target) {
                if (__hip_atomic_load(&sync->err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
                    ++spins > spin_limit) {
                    __hip_atomic_store(&sync->err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    abort_flag = 1;
                    break;
                }
                __builtin_amdgcn_s_sleep(2);
            }
        }
        __syncthreads();
        __threadfence();   // acquire: the other workgroups' stores of this pass
        if (abort_flag) break;
    }
}

hipError_t launch_persistent(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity0,
                             int npasses, int kind, int masked, SyncState* sync, uint64_t base, int spin_limit,
                             hipStream_t s)
{
    const int per = kBlock / kWave;
    const dim3 grid((ntiles + per - 1) / per);
    void* args[] = {(void*)&d_basins, (void*)&d_tiles, (void*)&ntiles, (void*)&parity0, (void*)&npasses,
                    (void*)&sync, (void*)&base, (void*)&spin_limit};
    if (kind == 2)
        return hipLaunchCooperativeKernel(masked ? (const void*)persistent_kernel<2, true>
                                                 : (const void*)persistent_kernel<2, false>,
                                          grid, dim3(kBlock), args, 0, s);
    if (masked)
        return hipLaunchCooperativeKernel((const void*)persistent_kernel<1, true>, grid, dim3(kBlock), args, 0, s);
    return hipLaunchCooperativeKernel((const void*)persistent_kernel<1, false>, grid, dim3(kBlock), args, 0, s);
}

int persistent_capacity(int kind, int masked, int ncu)
{
    int n = 0;
    if (kind == 2 && masked)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_kernel<2, true>, kBlock, 0);
    else if (kind == 2)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_kernel<2, false>, kBlock, 0);
    else if (masked)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_kernel<1, true>, kBlock, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, persistent_kernel<1, false>, kBlock, 0);
    return n * ncu;
}

}  // namespace mlb
