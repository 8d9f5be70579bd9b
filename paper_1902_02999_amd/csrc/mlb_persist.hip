// Persistent launches of the MacLABSWE step: many passes in one launch,
// separated by a cooperative grid barrier (persistent_kernel) or ordered per
// tile by a work queue with epoch flags (wq_kernel).
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

// Work-queue persistent kernel.  A grid of about one wave per tile of a pass
// (at most the resident capacity); each wave repeatedly takes the next (pass, tile) item from an atomic
// cursor, waits (bounded) until the tiles the item depends on have completed
// the previous pass (their epoch flags), runs the tile and publishes its own
// epoch.  Items are handed out in pass-major order, so every item an item
// waits for was handed out earlier to a running wave: the queue cannot
// deadlock, and the passes overlap instead of draining at a barrier.
// Release: the tile's stores are written back to the device level before the
// epoch store (agent-scope release fence); acquire: after the flags are seen,
// an agent-scope acquire fence before the tile's loads.  Waiting is bounded:
// with spin_limit polls, or once another wave has given up (err), a wave
// sets err and leaves; every wave then leaves at its next wait or item, so
// the grid drains (the state is then incomplete and the host reports it).
// A wait gives up after 2 s of the constant 100 MHz clock at most.
constexpr uint64_t kWqWaitTicks = 200000000ull;

template <int KIND, bool MASKED, bool CLOSED>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((KIND == 2 && CLOSED) ? 3 : 2)))
void wq_kernel(const BasinDev* __restrict__ basins, const TileDev* __restrict__ tiles, int ntiles, int parity0,
               int npasses, WorkQueue q, uint32_t epoch0, int spin_limit)
{
    // Every branch of the queue loop is on a wave-uniform value (read from
    // the first lane), so the loop is plain scalar control flow: the wave
    // takes an item, runs it and comes back for the next one, all lanes
    // together.
    const int lane = threadIdx.x & (kWave - 1);
    const uint32_t total = (uint32_t)ntiles * (uint32_t)npasses;
    // an earlier launch gave up: do nothing until the host has reset the state
    if (uniform(__hip_atomic_load(q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0) return;
    bool gave_up = false;
    for (;;) {
        uint32_t mine = 0;
        if (lane == 0) mine = __hip_atomic_fetch_add(q.cursor, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        const uint32_t i = (uint32_t)uniform((int)mine);   // lane 0's ticket
        if (i >= total) break;
        const int p = (int)(i / (uint32_t)ntiles), t = (int)(i - (uint32_t)p * (uint32_t)ntiles);
        if (p > 0) {
            // every dependency has completed pass p - 1 of this launch
            const uint32_t target = epoch0 + (uint32_t)p;
            const int b0 = uniform(q.nbr_off[t]), n = uniform(q.nbr_off[t + 1]) - b0;
            const int32_t dep = lane < n ? q.nbr[b0 + lane] : 0;
            const uint64_t t0 = (uint64_t)wall_clock64();
            int spins = 0;
            for (;;) {
                bool ready = true;
                if (lane < n) {
                    const uint32_t e = __hip_atomic_load(q.epoch + dep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    ready = (int32_t)(e - target) >= 0;
                }
                if (__all(ready)) break;
                // bounded in polls and in time (the constant clock), whichever
                // comes first; another wave's give-up is looked for every 16 polls
                int quit = (spins++ >= spin_limit || (uint64_t)wall_clock64() - t0 > kWqWaitTicks) ? 1 : 0;
                if (!quit && (spins & 15) == 0)
                    quit = uniform(__hip_atomic_load(q.err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) != 0;
                if (quit) { gave_up = true; break; }
                __builtin_amdgcn_s_sleep(2);
            }
            if (gave_up) break;
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
        } else if (spin_limit == 0 && npasses > 1) {
            // a wait limit of zero polls gives up at the first wait: with
            // more than one pass, the first wave to take an item gives up
            // (forces the give-up path from the host)
            gave_up = true;
            break;
        }
        const int64_t step = q.base[uniform(tiles[t].basin)] + (int64_t)p * KIND;
        pass_tile<KIND, false, MASKED, false, false, CLOSED>(basins, tiles, t, parity0 ^ (p & 1), nullptr,
                                                             FixedStep{step});
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
        if (lane == 0)
            __hip_atomic_store(q.epoch + t, epoch0 + (uint32_t)p + 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    if (gave_up && lane == 0) __hip_atomic_store(q.err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Before a work-queue launch: the cursor to 0 and every basin's step counter
// (at the parity the launch reads first) into q.base.
__global__ __launch_bounds__(kBlock) void wq_prologue_kernel(const BasinDev* __restrict__ basins, int nbasins,
                                                             int parity0, WorkQueue q)
{
    const int i = blockIdx.x * kBlock + threadIdx.x;
    if (i == 0) *q.cursor = 0u;
    if (i < nbasins) {
        const BasinDev& B = basins[i];
        q.base[i] = B.stepc[parity0 ^ B.swap];
    }
}

hipError_t launch_workqueue(const BasinDev* d_basins, int nbasins, const TileDev* d_tiles, int ntiles, int parity0,
                            int npasses, int kind, int masked, int closed, const WorkQueue& q, uint32_t epoch0,
                            int spin_limit, int nblocks, unsigned dyn_lds, hipStream_t s)
{
    hipLaunchKernelGGL(wq_prologue_kernel, dim3((nbasins + kBlock - 1) / kBlock), dim3(kBlock), 0, s, d_basins,
                       nbasins, parity0, q);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    using K = void (*)(const BasinDev*, const TileDev*, int, int, int, WorkQueue, uint32_t, int);
    static const K table[8] = {wq_kernel<1, false, false>, wq_kernel<1, false, false>,
                               wq_kernel<1, true, false>,  wq_kernel<1, true, false>,
                               wq_kernel<2, false, false>, wq_kernel<2, false, true>,
                               wq_kernel<2, true, false>,  wq_kernel<2, true, true>};
    hipLaunchKernelGGL(table[(kind == 2 ? 4 : 0) + (masked ? 2 : 0) + (closed ? 1 : 0)], dim3(nblocks), dim3(kBlock),
                       dyn_lds, s, d_basins, d_tiles, ntiles, parity0, npasses, q, epoch0, spin_limit);
    return hipGetLastError();
}

int workqueue_occupancy(int kind, int masked, int closed)
{
    using K = void (*)(const BasinDev*, const TileDev*, int, int, int, WorkQueue, uint32_t, int);
    static const K table[8] = {wq_kernel<1, false, false>, wq_kernel<1, false, false>,
                               wq_kernel<1, true, false>,  wq_kernel<1, true, false>,
                               wq_kernel<2, false, false>, wq_kernel<2, false, true>,
                               wq_kernel<2, true, false>,  wq_kernel<2, true, true>};
    int n = 0;
    (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, table[(kind == 2 ? 4 : 0) + (masked ? 2 : 0) + (closed ? 1 : 0)],
                                                      kBlock, 0);
    return n > 0 ? n : 1;
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
