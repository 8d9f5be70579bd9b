// gfx950 kernel of the MacLABSWE step with two steps per pass (temporal
// blocking; the walk is run_tile2 in mlb_step_impl.h) and its launcher.
#include "mlb_step_impl.h"

namespace mlb {

// One pass of two steps, over tiles of 60-column strips (MASKED: the list
// may hold TILE_MASKED tiles; CLOSED: walls and periodic edges only; IMPL:
// the implicit link depth, whose coefficients need more registers; DIAG: the
// second step is reduced into the tile's FP64 partials).
template <bool DIAG, bool MASKED, bool CLOSED, bool IMPL>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu((IMPL || (DIAG && MASKED)) ? 2 : 3)))
void step2_kernel(const BasinDev* __restrict__ basins, const TileDev* __restrict__ tiles, int ntiles,
                  int parity, double* __restrict__ partials)
{
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    pass_tile<2, DIAG, MASKED, IMPL, false, CLOSED>(basins, tiles, t, parity, partials, PlainStep{});
}

hipError_t launch_step2(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity,
                        double* d_partials, int diag, int masked, int implicit, int closed, unsigned dyn_lds,
                        hipStream_t s)
{
    const int per = kBlock / kWave;
    const dim3 grid((ntiles + per - 1) / per);
    using K2 = void (*)(const BasinDev*, const TileDev*, int, int, double*);
    static const K2 k2[16] = {
        step2_kernel<false, false, false, false>, step2_kernel<false, false, true, false>,
        step2_kernel<false, true, false, false>,  step2_kernel<false, true, true, false>,
        step2_kernel<false, false, false, true>,  step2_kernel<false, false, true, true>,
        step2_kernel<false, true, false, true>,   step2_kernel<false, true, true, true>,
        step2_kernel<true, false, false, false>,  step2_kernel<true, false, true, false>,
        step2_kernel<true, true, false, false>,   step2_kernel<true, true, true, false>,
        step2_kernel<true, false, false, true>,   step2_kernel<true, false, true, true>,
        step2_kernel<true, true, false, true>,    step2_kernel<true, true, true, true>};
    hipLaunchKernelGGL(k2[(diag ? 8 : 0) + (implicit ? 4 : 0) + (masked ? 2 : 0) + (closed ? 1 : 0)], grid,
                       dim3(kBlock), dyn_lds, s, d_basins, d_tiles, ntiles, parity, d_partials);
    return hipGetLastError();
}

}  // namespace mlb
