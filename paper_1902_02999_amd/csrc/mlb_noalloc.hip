// Allocation-free diagnostics (mlb_diag_noalloc): the FP64 mass / residual /
// max-speed / bad-node reduction of a grid written to a caller's device
// mlb_diag_t, for callers that cannot allocate device memory.
//
// The state reduction keeps its per-tile partial sums in `scratch`, a fixed
// device array of this file (one per GPU, held until the process ends).  Host
// code never passes the array's name to a kernel: at context set-up the
// device address of each GPU's copy is looked up once (noalloc_setup) and
// kept per device, and the kernels take that address as an argument.
#include <mutex>

#include "mlb_runtime.h"
#include "mlb_step_impl.h"

namespace mlb {

// Tiles of 64 columns x 64 rows; one partial set (kPartials doubles) each.
constexpr int kNaTile = 64;
constexpr int kNaMaxTiles = 16384;   // 16384 x 6 x 8 B = 768 KiB

static __device__ __align__(256) double scratch[kNaMaxTiles * kPartials];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_na_lock;
double* g_na_ptr[kMaxDevices] = {nullptr};   // each GPU's copy of `scratch`
}  // namespace

// Looks up this device's copy of the scratch array (the device must be
// current).  Called once per device by mlb_ctx_create.
mlb_status noalloc_setup(int device)
{
    if (device < 0 || device >= kMaxDevices) return fail(MLB_E_INVAL, "device index beyond the library's table");
    std::lock_guard<std::mutex> lk(g_na_lock);
    if (g_na_ptr[device]) return MLB_OK;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        return fail(MLB_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_na_ptr[device] = (double*)p;
    return MLB_OK;
}

// Fields of one grid as kernel arguments (no device descriptor).
struct NaFields {
    const float *eta, *qx, *qy, *qx0, *qy0, *H, *etal;
    const uint8_t* mask;
    int32_t nx, ny, ld, tiles_x;
};

// Wave t reduces tile (t % tiles_x, t / tiles_x): its lane's column over the
// tile's rows, with the checked pass's per-node arithmetic (account), into
// part[t].
__global__ __launch_bounds__(kBlock) void noalloc_reduce_kernel(NaFields F, int ntiles, double* __restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    const int x = (t % F.tiles_x) * kNaTile + lane;
    const int y0 = (t / F.tiles_x) * kNaTile, y1 = min(F.ny, y0 + kNaTile);
    Sums sums = {0.0, 0.0, 0.0, 0.0f, 0.0f};
    if (x < F.nx) {
        for (int r = y0; r < y1; ++r) {
            const size_t o = (size_t)r * F.ld + x;
            if (F.mask && F.mask[o] == NODE_SOLID) continue;   // not part of the water
            account(sums, F.eta[o], F.qx[o], F.qy[o], F.H[o], F.qx0[o], F.qy0[o], F.etal ? F.etal[o] : 0.0f);
        }
    }
    wave_partials(sums, part + (size_t)t * kPartials);
}

// Host-known constants of the diagnostics.
struct NaConsts {
    int64_t step;
    double dt, e, dx, nu, sumH, gh_over_e2;
};

// Sums the partials of `ntiles` tiles in a fixed order into the grid's result
// slot (ntiles == 0: the slot already holds the last checked pass's sums),
// then writes the caller's mlb_diag_t from the slot.
constexpr int kNaFin = 1024;
__global__ __launch_bounds__(kNaFin) void noalloc_finish_kernel(const double* __restrict__ part, int ntiles,
                                                                double* __restrict__ dres, NaConsts k,
                                                                mlb_diag_t* __restrict__ out)
{
    __shared__ double wsum[kNaFin / kWave][5];
    const int tid = threadIdx.x, lane = tid & (kWave - 1), w = tid >> 6;
    if (ntiles > 0) {
        double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
        for (int i = tid; i < ntiles; i += kNaFin) {
            const double* p = part + (size_t)i * kPartials;
            s[0] += p[0]; s[1] += p[1]; s[2] += p[2]; s[3] += p[3];
            s[4] = p[4] > s[4] ? p[4] : s[4];
        }
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
            for (int j = 0; j < 4; ++j) s[j] += __shfl_xor(s[j], off);
            const double vm = __shfl_xor(s[4], off);
            s[4] = vm > s[4] ? vm : s[4];
        }
        if (lane == 0)
            for (int j = 0; j < 5; ++j) wsum[w][j] = s[j];
        __syncthreads();
        if (tid == 0) {
            for (int v = 1; v < kNaFin / kWave; ++v) {
                for (int j = 0; j < 4; ++j) s[j] += wsum[v][j];
                s[4] = wsum[v][4] > s[4] ? wsum[v][4] : s[4];
            }
            for (int j = 0; j < 5; ++j) dres[j] = s[j];
            dres[5] = dres[6] = dres[7] = 0.0;
        }
    }
    if (tid == 0) {
        // the host's fill of mlb_diag, operation for operation
        const double s0 = dres[0], s1 = dres[1], s2 = dres[2], s3 = dres[3], s4 = dres[4];
        out->step = k.step;
        out->t = (double)k.step * k.dt;
        out->mass = (k.sumH + s0) * k.dx * k.dx;
        out->residual = s1 > 0 ? sqrt(s1) / sqrt(s2) : 0.0;
        out->max_speed = s4;
        out->nonfinite = (int64_t)s3;
        out->e = k.e;
        out->dt = k.dt;
        out->gh_over_e2 = k.gh_over_e2;
        out->rle = s4 * k.dx / k.nu;
    }
}

}  // namespace mlb

using namespace mlb;

extern "C" mlb_status mlb_diag_noalloc(mlb_grid* g, mlb_diag_t* out_dev)
{
    if (!g || !out_dev) return fail(MLB_E_INVAL, "grid or out_dev is NULL");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    mlb_ctx* c = g->ctx;
    const hipError_t de = hipSetDevice(c->device);
    if (de != hipSuccess) return fail(MLB_E_DEVICE, std::string("hipSetDevice: ") + hipGetErrorString(de));
    double* ptr = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_na_lock);
        ptr = c->device < kMaxDevices ? g_na_ptr[c->device] : nullptr;
    }
    if (!ptr) return fail(MLB_E_STATE, "the allocation-free scratch of this device was not set up");
    const int tx = (g->p.nx + kNaTile - 1) / kNaTile, ty = (g->p.ny + kNaTile - 1) / kNaTile;
    const int64_t ntiles = (int64_t)tx * ty;
    if (ntiles > kNaMaxTiles)
        return fail(MLB_E_INVAL, "grid too large for the allocation-free diagnostics: " + std::to_string(ntiles) +
                                     " tiles of 64 x 64 nodes, at most " + std::to_string(kNaMaxTiles));
    NaConsts k;
    k.step = g->step;
    k.dt = g->dt;
    k.e = g->e;
    k.dx = g->p.dx;
    k.nu = g->p.nu;
    k.sumH = g->sumH;
    k.gh_over_e2 = g->p.g * g->Hmax / (g->e * g->e);
    int nt = 0;
    if (!g->diag_fresh) {
        // the fields were set since the last checked pass: reduce the current
        // buffer against the other one (both hold the state: residual 0)
        const int cur = g->cur;
        NaFields F;
        F.eta = g->eta[cur]; F.qx = g->qx[cur]; F.qy = g->qy[cur];
        F.qx0 = g->qx[cur ^ 1]; F.qy0 = g->qy[cur ^ 1];
        F.H = g->H;
        F.etal = g->etal ? g->etal + (size_t)cur * g->plane : nullptr;
        F.mask = g->dmask;
        F.nx = g->p.nx; F.ny = g->p.ny; F.ld = g->ld; F.tiles_x = tx;
        const int per = kBlock / kWave;
        hipLaunchKernelGGL(noalloc_reduce_kernel, dim3((unsigned)((ntiles + per - 1) / per)), dim3(kBlock), 0,
                           c->stream, F, (int)ntiles, ptr);
        const hipError_t e = hipGetLastError();
        if (e != hipSuccess) return fail(MLB_E_DEVICE, std::string("noalloc_reduce_kernel: ") + hipGetErrorString(e));
        nt = (int)ntiles;
    }
    hipLaunchKernelGGL(noalloc_finish_kernel, dim3(1), dim3(kNaFin), 0, c->stream, (const double*)ptr, nt, g->dres,
                       k, out_dev);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(MLB_E_DEVICE, std::string("noalloc_finish_kernel: ") + hipGetErrorString(e));
    g->diag_fresh = true;
    return MLB_OK;
}
