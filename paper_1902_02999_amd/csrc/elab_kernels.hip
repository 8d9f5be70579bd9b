// gfx950 kernel of the eLABSWE baseline (Zhou, arXiv 1902.02999, Eq. lb.1):
// nine stored FP32 distributions per node relaxed with a single time tau and
// streamed, the lattice Boltzmann equation the streaming-only method is
// derived from.  It exists to measure, on the same hardware and tiles, what
// storing distributions costs against the three macroscopic fields of the
// streaming-only step.
//
// Per node x, upstream neighbours y_a = x - e_a dt (pull form, Eq. lb.Mac.1):
//   f*_a(n)   = f_a(n) + (f_a^eq(n) - f_a(n)) / tau            (collision at n)
//   f_a(x)'   = f*_a(y_a) - g/(2e^2) C_a (h_x + h_y)(H_y - H_x)
//               + C_a e^_a . (Fp(x) + Fp(y_a)),   Fp = dt F / (2e)
// with Eq. feq-full for f^eq, the old-time link depth of Eq. h-bar and the
// link-midpoint force of Eq. force-CS (z_x - z_y = H_y - H_x).  A link whose
// upstream node is past a wall edge or SOLID takes f*_abar(x) and no bed or
// force term; nodes on wall edges and WALL nodes end at f^eq(h', 0); SOLID
// nodes are never written.  Open edges are not supported by this baseline.
//
// Stored variable: g_a = f_a - w_a(H), the distributions minus the node's
// still-water equilibrium w_a(H) = f_a^eq(H, 0) (static).  The map is the same
// in exact arithmetic; in FP32 it avoids cancelling O(g H^2 / e^2) parts:
//   eta = sum_a g_a, q = e sum_a e^_a g_a (w_a is even in e^_a),
//   g_a^eq = f_a^eq(h, u) - w_a(H), whose hydrostatic part is
//            C_a g eta (h + H) / (2 e^2) (a != 0),
//   g_a(x)' = g*_a(y) - g/(2e^2) C_a (H_y - H_x)(eta_x + eta_y) + C_a e^_a . (Fp(x) + Fp(y)),
// the middle term being the bed term plus w_a(H_y) - w_a(H_x); it vanishes for
// still water at the reference level, so still water stays still exactly.
// Bounced links take g*_abar(x) (w_abar = w_a).
//
// Execution mirrors the streaming-only one-step kernel: one wave per tile of
// 62 output columns (lanes 0 and 63 are the halo), rows walked with a
// three-row register window, lane neighbours through DPP shifts.  Each row
// loads its nine distributions and H once (40 B per node, plus the kind byte
// in masked tiles) and each owned node stores nine (36 B).
#include "mlb_internal.h"

// Build-time knob (results are bitwise independent of it):
//   MLB_ELAB_NT_STORE  non-temporal stores of the new distributions (off:
//                      with nine store streams per wave they were measured
//                      14 % slower on MI355X than ordinary stores)
#ifndef MLB_ELAB_NT_STORE
#define MLB_ELAB_NT_STORE 0
#endif

namespace mlb {
namespace elab {

__device__ __forceinline__ float from_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x138, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(__builtin_bit_cast(int, v), 0x130, 0xf, 0xf, true));
}
__device__ __forceinline__ int from_left_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x138, 0xf, 0xf, true); }
__device__ __forceinline__ int from_right_i(int v) { return __builtin_amdgcn_mov_dpp(v, 0x130, 0xf, 0xf, true); }
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

__device__ __forceinline__ int wrap_or_clamp(int r, int n, int periodic)
{
    if (periodic) {
        const int m = r % n;
        return m < 0 ? m + n : m;
    }
    return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

// D2Q9 numbering of the paper's Section 3 as used throughout: direction a
// has e^_a = (EX[a], EY[a]); odd directions are axes (C = 1/3, lambda = 1),
// even ones diagonals (C = 1/12, lambda = 1/4); OPP[a] is the reverse.
constexpr int EX[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
constexpr int EY[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
constexpr int OPP[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};
__device__ __forceinline__ constexpr float cof(int a) { return a == 0 ? 0.0f : (a & 1 ? 1.0f / 3.0f : 1.0f / 12.0f); }
__device__ __forceinline__ constexpr float lam(int a) { return a & 1 ? 1.0f : 0.25f; }

// What a row of the window holds per lane: post-collision deviations g*,
// surface perturbation, still-water depth, half-step force, node kind and
// SOLID bits.
struct ERow {
    float fs[9];
    float eta, H, fpx, fpy;
    int mk, ms;
};

// g_a^eq = f_a^eq(h, u) - w_a(H) (Eq. feq-full minus the still-water part).
__device__ __forceinline__ float geq(const ElabDev& D, int a, float eta, float h, float H, float u, float v)
{
    const float uu = __builtin_fmaf(u, u, v * v);
    const float hyd = D.g6 * eta * (h + H);     // g (h^2 - H^2) / (6 e^2)
    if (a == 0) return __builtin_fmaf(-5.0f, hyd, eta) - 4.0f * D.c6 * h * uu;
    const float eu = (float)EX[a] * u + (float)EY[a] * v;
    // lambda_a [g (h^2 - H^2)/(6e^2) + h (e^.u/(3e) + (e^.u)^2/(2e^2) - |u|^2/(6e^2))]
    return lam(a) * __builtin_fmaf(h, __builtin_fmaf(eu, __builtin_fmaf(D.c2, eu, D.c3), -D.c6 * uu), hyd);
}

template <bool FRIC>
__device__ __forceinline__ void collide(const ElabDev& D, const float* f, float H, ERow& R)
{
    float eta = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        eta += f[a];
        if (EX[a]) sx += EX[a] > 0 ? f[a] : -f[a];
        if (EY[a]) sy += EY[a] > 0 ? f[a] : -f[a];
    }
    const float h = H + eta;
    const float qx = D.e * sx, qy = D.e * sy;
    const float r = __builtin_amdgcn_rcpf(h);
    const float u = qx * r, v = qy * r;
    // Fp = dt/(2e) [tau_w/rho - C_b u |u| + Omega (qy, -qx)]
    float fx = D.tx, fy = D.ty;
    if (FRIC) {
        const float s = __builtin_amdgcn_sqrtf(__builtin_fmaf(u, u, v * v));
        fx = __builtin_fmaf(-D.cb * s, u, fx);
        fy = __builtin_fmaf(-D.cb * s, v, fy);
    }
    fx = __builtin_fmaf(D.om, qy, fx);
    fy = __builtin_fmaf(-D.om, qx, fy);
    R.fpx = D.cfp * fx;
    R.fpy = D.cfp * fy;
#pragma unroll
    for (int a = 0; a < 9; ++a) R.fs[a] = __builtin_fmaf(D.rtau, geq(D, a, eta, h, H, u, v) - f[a], f[a]);
    R.eta = eta;
    R.H = H;
}

__device__ __forceinline__ void kinds(int m, ERow& R)
{
    const int s = m == NODE_SOLID ? 1 : 0;
    R.mk = m;
    R.ms = from_left_i(s) | (s << 1) | (from_right_i(s) << 2);
}

// The upstream row values of link a for the node at this lane.
struct Up { float fs, eta, H, fpx, fpy; };

template <int A>
__device__ __forceinline__ Up upstream(const ERow& S, const ERow& C, const ERow& N)
{
    // row of y_a = x - e_a: EY = +1 -> row below (S), -1 -> row above (N)
    const ERow& R = EY[A] > 0 ? S : (EY[A] < 0 ? N : C);
    Up u;
    if (EX[A] > 0) {        // y at x - 1
        u.fs = from_left(R.fs[A]); u.eta = from_left(R.eta); u.H = from_left(R.H);
        u.fpx = from_left(R.fpx); u.fpy = from_left(R.fpy);
    } else if (EX[A] < 0) { // y at x + 1
        u.fs = from_right(R.fs[A]); u.eta = from_right(R.eta); u.H = from_right(R.H);
        u.fpx = from_right(R.fpx); u.fpy = from_right(R.fpy);
    } else {
        u.fs = R.fs[A]; u.eta = R.eta; u.H = R.H; u.fpx = R.fpx; u.fpy = R.fpy;
    }
    return u;
}

template <int A>
__device__ __forceinline__ float stream(const ElabDev& D, const ERow& S, const ERow& C, const ERow& N, bool bounce)
{
    const Up y = upstream<A>(S, C, N);
    const float bed = -D.gb * cof(A) * ((y.H - C.H) * (C.eta + y.eta));
    const float frc = cof(A) * ((float)EX[A] * (C.fpx + y.fpx) + (float)EY[A] * (C.fpy + y.fpy));
    const float v = (y.fs + bed) + frc;
    return bounce ? C.fs[OPP[A]] : v;
}

typedef __attribute__((address_space(1))) const float gcf;
typedef __attribute__((address_space(1))) float gf;

struct Raw { float f[9]; float H; int m; };

// Plane bases of one buffer (uniform) and the 32-bit element offset of a row.
struct Planes { const gcf* p[9]; };

template <bool MASK>
__device__ __forceinline__ void load_row(const ElabDev& D, const Planes& F, uint32_t o, Raw& w)
{
#pragma unroll
    for (int a = 0; a < 9; ++a) w.f[a] = F.p[a][o];
    w.H = ((gcf*)D.H)[o];
    w.m = MASK ? (int)D.mask[o] : 0;
}

struct Lane { int x; bool own_col, wout, eout; };

// Output row r from window rows S (r-1), C (r), N (r+1); N is formed here from
// the raw row w, which is then refilled with row `next` (three rows ahead).
template <bool EDGE, bool MASK, bool FRIC>
__device__ __forceinline__ void row_step(const ElabDev& D, const Planes& F, gf* const* G, const Lane& L,
                                         const TileDev& T, int r, int r1, const ERow& S, const ERow& C, ERow& N,
                                         Raw& w, uint32_t next)
{
    collide<FRIC>(D, w.f, w.H, N);
    if (MASK) kinds(w.m, N);
    load_row<MASK>(D, F, next, w);
    const bool sout = EDGE && !D.per_y && r == 0, nout = EDGE && !D.per_y && r == D.ny - 1;
    bool b[9] = {false, L.wout, L.wout || sout, sout, L.eout || sout, L.eout, L.eout || nout, nout, L.wout || nout};
    if (MASK) {
        b[1] = b[1] || (C.ms & 1); b[5] = b[5] || (C.ms & 4);
        b[2] = b[2] || (S.ms & 1); b[3] = b[3] || (S.ms & 2); b[4] = b[4] || (S.ms & 4);
        b[8] = b[8] || (N.ms & 1); b[7] = b[7] || (N.ms & 2); b[6] = b[6] || (N.ms & 4);
    }
    float fn[9];
    fn[0] = C.fs[0];
    fn[1] = stream<1>(D, S, C, N, b[1]);
    fn[2] = stream<2>(D, S, C, N, b[2]);
    fn[3] = stream<3>(D, S, C, N, b[3]);
    fn[4] = stream<4>(D, S, C, N, b[4]);
    fn[5] = stream<5>(D, S, C, N, b[5]);
    fn[6] = stream<6>(D, S, C, N, b[6]);
    fn[7] = stream<7>(D, S, C, N, b[7]);
    fn[8] = stream<8>(D, S, C, N, b[8]);
    const bool wall = (EDGE && (L.wout || L.eout || sout || nout)) || (MASK && C.mk == NODE_WALL);
    if (wall) {
        // zero-velocity equilibrium at the new depth (q = 0 on walls)
        float eta = 0.0f;
#pragma unroll
        for (int a = 0; a < 9; ++a) eta += fn[a];
        const float hyd = D.g6 * eta * ((C.H + eta) + C.H);
        fn[0] = __builtin_fmaf(-5.0f, hyd, eta);
#pragma unroll
        for (int a = 1; a < 9; ++a) fn[a] = lam(a) * hyd;
    }
    if (L.own_col && r >= T.yo && r < r1 && !(MASK && C.mk == NODE_SOLID)) {
        const uint32_t o = (uint32_t)r * (uint32_t)D.ld + (uint32_t)L.x;
#pragma unroll
        for (int a = 0; a < 9; ++a) {
#if MLB_ELAB_NT_STORE
            __builtin_nontemporal_store(fn[a], &G[a][o]);
#else
            G[a][o] = fn[a];
#endif
        }
    }
}

template <bool EDGE, bool MASK, bool FRIC>
__device__ void run_tile(const ElabDev& D, const TileDev T, int rd)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = D.nx, ny = D.ny;
    Lane L;
    L.x = T.x0 + lane - 1;
    const int xl = wrap_or_clamp(L.x, nx, D.per_x);
    L.own_col = lane >= 1 && lane <= kStripOut && L.x >= T.xo && L.x < nx;
    L.wout = EDGE && !D.per_x && L.x == 0;
    L.eout = EDGE && !D.per_x && L.x == nx - 1;
    Planes F;
    gf* G[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        F.p[a] = (const gcf*)D.f[rd] + (size_t)a * D.plane;
        G[a] = (gf*)D.f[rd ^ 1] + (size_t)a * D.plane;
    }
    const int r0 = T.y0, r1 = T.y0 + T.rows;
    auto off = [&](int r) { return (uint32_t)wrap_or_clamp(min(r, r1), ny, D.per_y) * (uint32_t)D.ld + (uint32_t)xl; };
    // rows are loaded three rows before they are collided; the window and the
    // raw slots rotate with period 3, so the loop is unrolled by 3
    ERow R0, R1, R2;
    Raw wa, wb, wc;
    load_row<MASK>(D, F, off(r0 - 1), wa);
    collide<FRIC>(D, wa.f, wa.H, R0);
    if (MASK) kinds(wa.m, R0);
    load_row<MASK>(D, F, off(r0), wa);
    collide<FRIC>(D, wa.f, wa.H, R1);
    if (MASK) kinds(wa.m, R1);
    load_row<MASK>(D, F, off(r0 + 1), wa);
    load_row<MASK>(D, F, off(r0 + 2), wb);
    load_row<MASK>(D, F, off(r0 + 3), wc);
    const int nk = (T.rows + 2) / 3;
    int r = r0;
    for (int k = 0; k < nk; ++k) {
        row_step<EDGE, MASK, FRIC>(D, F, G, L, T, r, r1, R0, R1, R2, wa, off(r + 4));
        ++r;
        row_step<EDGE, MASK, FRIC>(D, F, G, L, T, r, r1, R1, R2, R0, wb, off(r + 4));
        ++r;
        row_step<EDGE, MASK, FRIC>(D, F, G, L, T, r, r1, R2, R0, R1, wc, off(r + 4));
        ++r;
    }
}

__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(3)))
void elab_step_kernel(const ElabDev D, const TileDev* __restrict__ tiles, int ntiles, int rd)
{
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    const TileDev T = tiles[t];
    const bool edge = (!D.per_x && (T.x0 == 0 || T.x0 + kStripOut >= D.nx)) ||
                      (!D.per_y && (T.y0 == 0 || T.y0 + T.rows >= D.ny));
    const bool masked = (T.flags & TILE_MASKED) != 0;
    if (D.cb != 0.0f) {
        if (masked) run_tile<true, true, true>(D, T, rd);
        else if (edge) run_tile<true, false, true>(D, T, rd);
        else run_tile<false, false, true>(D, T, rd);
    } else {
        if (masked) run_tile<true, true, false>(D, T, rd);
        else if (edge) run_tile<true, false, false>(D, T, rd);
        else run_tile<false, false, false>(D, T, rd);
    }
}

// f := f^eq(h, q) of a macroscopic state (eta, qx, qy with h = H + eta), both buffers.
__global__ __launch_bounds__(kBlock) void elab_init_kernel(const ElabDev D, const float* __restrict__ eta,
                                                           const float* __restrict__ qx,
                                                           const float* __restrict__ qy)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= D.nx || j >= D.ny) return;
    const size_t o = (size_t)j * D.ld + i;
    const float H = D.H[o], e = eta[o], h = H + e;
    const float r = 1.0f / h, u = qx[o] * r, v = qy[o] * r;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const float g = geq(D, a, e, h, H, u, v);
        D.f[0][(size_t)a * D.plane + o] = g;
        D.f[1][(size_t)a * D.plane + o] = g;
    }
}

// h - H, hu, hv of the distributions in buffer rd (Eqs. fea-0-h, fea-0-v):
// sums of the stored deviations.
__global__ __launch_bounds__(kBlock) void elab_macro_kernel(const ElabDev D, int rd, float* __restrict__ eta,
                                                            float* __restrict__ qx, float* __restrict__ qy)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= D.nx || j >= D.ny) return;
    const size_t o = (size_t)j * D.ld + i;
    float f[9];
#pragma unroll
    for (int a = 0; a < 9; ++a) f[a] = D.f[rd][(size_t)a * D.plane + o];
    float h = 0.0f, sx = 0.0f, sy = 0.0f;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        h += f[a];
        if (EX[a]) sx += EX[a] > 0 ? f[a] : -f[a];
        if (EY[a]) sy += EY[a] > 0 ? f[a] : -f[a];
    }
    eta[o] = h;
    qx[o] = D.e * sx;
    qy[o] = D.e * sy;
}

// The distributions f_a = g_a + w_a(H) of buffer rd into out [9][ny][nx].
__global__ __launch_bounds__(kBlock) void elab_dist_kernel(const ElabDev D, int rd, float* __restrict__ out)
{
    const int i = blockIdx.x * blockDim.x + threadIdx.x, j = blockIdx.y;
    if (i >= D.nx || j >= D.ny) return;
    const size_t o = (size_t)j * D.ld + i, n = (size_t)D.nx * D.ny, d = (size_t)j * D.nx + i;
    const float H = D.H[o], hs = D.g6 * H * H;
#pragma unroll
    for (int a = 0; a < 9; ++a) {
        const float w = a == 0 ? H - 5.0f * hs : lam(a) * hs;
        out[(size_t)a * n + d] = D.f[rd][(size_t)a * D.plane + o] + w;
    }
}

}  // namespace elab

hipError_t launch_elab_dist(const ElabDev& D, int rd, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(elab::elab_dist_kernel, dim3((D.nx + kBlock - 1) / kBlock, D.ny), dim3(kBlock), 0, s, D,
                       rd, out);
    return hipGetLastError();
}

hipError_t launch_elab_step(const ElabDev& D, const TileDev* d_tiles, int ntiles, int rd, hipStream_t s)
{
    const int per = kBlock / kWave;
    hipLaunchKernelGGL(elab::elab_step_kernel, dim3((ntiles + per - 1) / per), dim3(kBlock), 0, s, D, d_tiles,
                       ntiles, rd);
    return hipGetLastError();
}

hipError_t launch_elab_init(const ElabDev& D, const float* eta, const float* qx, const float* qy, hipStream_t s)
{
    hipLaunchKernelGGL(elab::elab_init_kernel, dim3((D.nx + kBlock - 1) / kBlock, D.ny), dim3(kBlock), 0, s, D,
                       eta, qx, qy);
    return hipGetLastError();
}

hipError_t launch_elab_macro(const ElabDev& D, int rd, float* eta, float* qx, float* qy, hipStream_t s)
{
    hipLaunchKernelGGL(elab::elab_macro_kernel, dim3((D.nx + kBlock - 1) / kBlock, D.ny), dim3(kBlock), 0, s, D,
                       rd, eta, qx, qy);
    return hipGetLastError();
}

}  // namespace mlb
