// gfx950 kernels of the MacLABSWE streaming-only step (Zhou, arXiv 1902.02999):
// one step per pass, persistent launches, reductions, the copy probe and the
// host-side launchers.  The per-node arithmetic and the tile walks are in
// mlb_step_impl.h; the two-step kernel is in mlb_kernels2.hip.
#include "mlb_step_impl.h"

namespace mlb {

// One pass of one step.  One wave per tile, tiles in list order (largest
// basins first): the hardware dispatcher hands out workgroups in index
// order, so the list is consumed as a queue without a software loop.
// (two or more of the checked step, the mask, the implicit link depth and
// the compensated surface together need more than 128 VGPRs)
template <bool DIAG, bool MASKED, bool IMPL, bool COMP>
__global__ __launch_bounds__(kBlock)
__attribute__((amdgpu_waves_per_eu((int(DIAG) + int(MASKED) + int(IMPL) + int(COMP) >= 2) ? 3 : 4)))
void step_kernel(const BasinDev* __restrict__ basins, const TileDev* __restrict__ tiles, int ntiles,
                 int parity, double* __restrict__ partials)
{
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    pass_tile<1, DIAG, MASKED, IMPL, COMP, false>(basins, tiles, t, parity, partials, PlainStep{});
}


// Reduction of the current state (no step): same partial layout and the
// same per-node arithmetic as the checked pass (account).
__global__ __launch_bounds__(kBlock) void reduce_state_kernel(const BasinDev* __restrict__ basins,
                                                              const TileDev* __restrict__ tiles,
                                                              int ntiles, int parity,
                                                              double* __restrict__ partials)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    const TileDev T = tiles[t];
    const BasinDev& B = basins[T.basin];
    const int cur = parity ^ B.swap, prev = cur ^ 1;
    const int x = T.x0 + lane - 1;
    const bool own_col = lane >= 1 && lane <= kStripOut && x >= T.xo && x < B.nx;
    Sums sums = {0.0, 0.0, 0.0, 0.0f, 0.0f};
    if (own_col) {
        for (int r = T.yo; r < T.y0 + T.rows; ++r) {
            const size_t o = (size_t)r * B.ld + x;
            if (B.mask && B.mask[o] == NODE_SOLID) continue;   // not part of the water
            const float el = B.etal[cur] ? B.etal[cur][o] : 0.0f;   // compensated surface
            account(sums, B.eta[cur][o], B.qx[cur][o], B.qy[cur][o], B.H[o], B.qx[prev][o], B.qy[prev][o], el);
        }
    }
    wave_partials(sums, partials + (size_t)t * kPartials);
}

// Per-basin sum of the tile partials in a fixed order: thread i of the block
// sums tiles i, i + kFinBlock, ... of the basin in that order, then a fixed
// butterfly across each wave and the waves' results in order.
constexpr int kFinBlock = 1024;
__global__ __launch_bounds__(kFinBlock) void finalize_kernel(const BasinDev* __restrict__ basins,
                                                             const double* __restrict__ partials,
                                                             double* __restrict__ out, int kind)
{
    __shared__ double wsum[kFinBlock / kWave][5];
    const BasinDev& B = basins[blockIdx.x];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid >> 6;
    // partials of a one-step pass (or of the state reduction) are indexed by the
    // one-step tile list, those of a two-step pass by the two-step list
    const int first = kind == 2 ? B.first_tile2 : B.first_tile, nt = kind == 2 ? B.ntiles2 : B.ntiles;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    // four tiles' loads in flight at once, added in tile order
    int i = tid;
    for (; i + 3 * kFinBlock < nt; i += 4 * kFinBlock) {
        double v[4][5];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const double* p = partials + (size_t)(first + i + u * kFinBlock) * kPartials;
#pragma unroll
            for (int k = 0; k < 5; ++k) v[u][k] = p[k];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            s[0] += v[u][0]; s[1] += v[u][1]; s[2] += v[u][2]; s[3] += v[u][3];
            s[4] = v[u][4] > s[4] ? v[u][4] : s[4];
        }
    }
    for (; i < nt; i += kFinBlock) {
        const double* p = partials + (size_t)(first + i) * kPartials;
        s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] += p[3];
        s[4] = p[4] > s[4] ? p[4] : s[4];
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int k = 0; k < 4; ++k) s[k] += __shfl_xor(s[k], off);
        const double vm = __shfl_xor(s[4], off);
        s[4] = vm > s[4] ? vm : s[4];
    }
    if (lane == 0)
        for (int k = 0; k < 5; ++k) wsum[w][k] = s[k];
    __syncthreads();
    if (tid == 0) {
        for (int v = 1; v < kFinBlock / kWave; ++v) {
            for (int k = 0; k < 4; ++k) s[k] += wsum[v][k];
            s[4] = wsum[v][4] > s[4] ? wsum[v][4] : s[4];
        }
        double* o = out + (size_t)blockIdx.x * 8;
        o[0] = s[0]; o[1] = s[1]; o[2] = s[2]; o[3] = s[3]; o[4] = s[4];
        o[5] = (double)B.stepc[0]; o[6] = (double)B.stepc[1]; o[7] = 0.0;
        if (B.dres)   // the basin's own copy, kept with its fields
            for (int k = 0; k < 8; ++k) B.dres[k] = o[k];
    }
}

// Plain device-to-device copy (16-byte vectors, grid-stride): the reference
// for the practical HBM bandwidth and for scaling the HBM byte counters.
__global__ __launch_bounds__(kBlock) void copy_probe_kernel(const float4* __restrict__ a,
                                                           float4* __restrict__ b, size_t n)
{
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) b[i] = a[i];
}

// ------------------------------------------------------------------ launchers
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL(copy_probe_kernel, dim3(nblocks), dim3(kBlock), 0, s, (const float4*)src,
                       (float4*)dst, bytes / sizeof(float4));
    return hipGetLastError();
}

int step_occupancy(int diag)
{
    int n = 0;
    if (diag)
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<true, false, false, false>, kBlock, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<false, false, false, false>, kBlock, 0);
    return n > 0 ? n : 1;
}

template <bool DIAG, bool MASKED, bool IMPL, bool COMP>
static void launch_one(dim3 grid, unsigned dyn_lds, hipStream_t s, const BasinDev* d_basins, const TileDev* d_tiles,
                       int ntiles, int parity, double* d_partials)
{
    hipLaunchKernelGGL((step_kernel<DIAG, MASKED, IMPL, COMP>), grid, dim3(kBlock), dyn_lds, s, d_basins, d_tiles,
                       ntiles, parity, d_partials);
}

hipError_t launch_step(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity,
                       double* d_partials, int diag, int tblock, int masked, int implicit, int comp,
                       int closed, unsigned dyn_lds, hipStream_t s)
{
    // dyn_lds: unused dynamic LDS that caps resident workgroups per CU
    if (tblock != 1 && (tblock != 2 || comp)) return hipErrorInvalidValue;
    if (tblock == 2)
        return launch_step2(d_basins, d_tiles, ntiles, parity, d_partials, diag, masked, implicit, closed, dyn_lds, s);
    const int per = kBlock / kWave;
    const dim3 grid((ntiles + per - 1) / per);
    using L = void (*)(dim3, unsigned, hipStream_t, const BasinDev*, const TileDev*, int, int, double*);
    static const L table[16] = {
        launch_one<false, false, false, false>, launch_one<false, false, false, true>,
        launch_one<false, false, true, false>,  launch_one<false, false, true, true>,
        launch_one<false, true, false, false>,  launch_one<false, true, false, true>,
        launch_one<false, true, true, false>,   launch_one<false, true, true, true>,
        launch_one<true, false, false, false>,  launch_one<true, false, false, true>,
        launch_one<true, false, true, false>,   launch_one<true, false, true, true>,
        launch_one<true, true, false, false>,   launch_one<true, true, false, true>,
        launch_one<true, true, true, false>,    launch_one<true, true, true, true>};
    table[(diag ? 8 : 0) + (masked ? 4 : 0) + (implicit ? 2 : 0) + (comp ? 1 : 0)](grid, dyn_lds, s, d_basins,
                                                                                   d_tiles, ntiles, parity,
                                                                                   d_partials);
    return hipGetLastError();
}

hipError_t launch_reduce_state(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles,
                               int parity, double* d_partials, hipStream_t s)
{
    const int per = kBlock / kWave;
    hipLaunchKernelGGL(reduce_state_kernel, dim3((ntiles + per - 1) / per), dim3(kBlock), 0, s,
                       d_basins, d_tiles, ntiles, parity, d_partials);
    return hipGetLastError();
}

hipError_t launch_finalize(const BasinDev* d_basins, int nbasins, const double* d_partials,
                           double* d_out, int kind, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(nbasins), dim3(kFinBlock), 0, s, d_basins, d_partials, d_out, kind);
    return hipGetLastError();
}

}  // namespace mlb
