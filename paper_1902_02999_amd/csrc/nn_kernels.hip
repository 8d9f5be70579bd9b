// gfx950 kernels of the warm-start network: 3x3 convolutions as implicit
// GEMMs on BF16 MFMA (v_mfma_f32_16x16x32_bf16, FP32 accumulation), the
// weight gradient with a deterministic split-K, pooling / upsampling, the 1x1
// head, the masked MSE loss and AdamW.
//
// Layouts: activations NHWC BF16 with a channel stride `ld` and offset (so a
// concatenation is just two writers into one buffer); gradients NHWC FP32;
// conv weights [Cout][9][Cin] BF16 (tap = 3 dy + dx), which is also the order
// of the FP32 master parameters.
//
// MFMA 16x16x32 operand layout (64 lanes; l16 = lane % 16, lq = lane / 16):
//   A (16 x 32):  lane holds A[l16][8 lq .. 8 lq + 7]
//   B (32 x 16):  lane holds B[8 lq .. 8 lq + 7][l16]
//   D (16 x 16):  lane holds D[4 lq .. 4 lq + 3][l16]
#include <algorithm>
#include <cmath>

#include "nn_internal.h"

namespace mlb {
namespace nn {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x4 __attribute__((ext_vector_type(4)));
typedef unsigned short u16x8 __attribute__((ext_vector_type(8)));

__device__ __forceinline__ f32x4 mfma(const bf16x8& a, const bf16x8& b, const f32x4& c)
{
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 load8(const __bf16* p)  // 16-byte aligned
{
    return *(const bf16x8*)p;
}

__device__ __forceinline__ bf16x8 zero8()
{
    bf16x8 z;
#pragma unroll
    for (int e = 0; e < 8; ++e) z[e] = (__bf16)0.0f;
    return z;
}

// ------------------------------------------------------------------ conv 3x3
// Y[p][n] = act(bias[n] + sum_{t,c} X[p + off_t][c] W[n][t][c]) as an
// implicit GEMM on MFMA.  A workgroup of eight waves computes kConvRows image
// rows (one per wave) of PT = 16 MB pixels x NT = 16 NB output channels (MB,
// NB in {2, 4}: each A fragment serves NB products and each B fragment MB).
// Per block of 32 input channels the workgroup stages the rows' input with
// its one-pixel halo, (kConvRows + 2) x (PT + 2) x 32 values (zero outside
// the image), and the NT x 9 x 32 weights in LDS; the nine taps then read
// their shifted A fragments and their B fragments from there instead of from
// global memory.  Each thread fetches its share of a block (a fixed number of
// 16-byte chunks) with all loads in flight at once, into registers, and
// writes them to LDS; with PF the fetch of block k + 1 is issued right after
// block k is in LDS, so it runs under block k's MFMAs (one LDS buffer: the
// registers carry the next block across the barrier).  Every output sums
// over channel blocks, then taps, in that order, whatever PF.  OUT_F32: FP32
// output (optionally accumulated into), else BF16.
constexpr int kConvRows = 8;               // one wave per row: kConvRows x 64 threads
constexpr int kConvThreads = kConvRows * 64;
// LDS elements per staged pixel: 32 channels + 8 of padding.  With 80-byte
// pixels the 16-byte A-fragment reads of neighbouring pixels start in
// distinct banks (64-byte pixels put every fourth pixel on the same banks).
constexpr int kConvPix = 40;
// The dispatcher deals workgroups to the eight XCDs in turn.  Block b of a
// grid of 8 k blocks takes list entry (b % 8) k + b / 8, so XCD j runs the
// j-th eighth of the list and neighbouring entries (which share input data)
// share one L2; blocks past 8 k keep their own index.
__device__ __forceinline__ int xcd_block(int b, int nblocks)
{
    const int per = nblocks / 8;
    return b < per * 8 ? (b % 8) * per + b / 8 : b;
}

template <bool OUT_F32, int MB, int NB, bool PF>
__global__ __launch_bounds__(kConvThreads) void conv3x3_lds_kernel(ConvArgs a)
{
    constexpr int PT = 16 * MB, NT = 16 * NB, TW = PT + 2;
    constexpr int CHUNKS = (kConvRows + 2) * TW * 4;   // 16-byte chunks of 8 channels
    constexpr int WS = 9 * 32 + 8;                    // per output channel: 9 taps x 32 inputs, padded
    constexpr int WCHUNKS = NT * 9 * 4;
    constexpr int XPT = (CHUNKS + kConvThreads - 1) / kConvThreads;    // input chunks per thread
    constexpr int WPT = (WCHUNKS + kConvThreads - 1) / kConvThreads;   // weight chunks per thread
    __shared__ __attribute__((aligned(16))) __bf16 tile[(kConvRows + 2) * TW * kConvPix];
    __shared__ __attribute__((aligned(16))) __bf16 wtile[NT * WS];
    const int wv = threadIdx.x >> 6, lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
    const int ntile = a.cout / NT, xtiles = a.w / PT, ygroups = (a.h + kConvRows - 1) / kConvRows;
    // (image, row group, pixel tile, channel tile), channels fastest; the
    // channel tiles of one input tile run on one XCD
    int b = xcd_block(blockIdx.x, gridDim.x);
    const int nt = b % ntile; b /= ntile;
    const int xt = b % xtiles; b /= xtiles;
    const int yg = b % ygroups;
    const int img = b / ygroups;
    const int x0 = xt * PT, n0 = nt * NT, y0 = yg * kConvRows;
    const int y = y0 + wv;
    const bool active = y < a.h;            // every wave still takes part in the loads and barriers

    f32x4 acc[MB][NB];
#pragma unroll
    for (int i = 0; i < MB; ++i)
#pragma unroll
        for (int j = 0; j < NB; ++j) acc[i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    bf16x8 xr[XPT], wr[WPT];
    auto fetch = [&](int c0) {
#pragma unroll
        for (int j = 0; j < XPT; ++j) {
            const int i = threadIdx.x + j * kConvThreads;
            xr[j] = zero8();
            if (i < CHUNKS) {
                const int ch8 = i & 3, px = (i >> 2) % TW, rr = (i >> 2) / TW;
                const int yy = y0 + rr - 1, xx = x0 + px - 1;
                if (yy >= 0 && yy < a.h && xx >= 0 && xx < a.w) {
                    const size_t src = a.up ? ((size_t)img * (a.h >> 1) + (yy >> 1)) * (a.w >> 1) + (xx >> 1)
                                            : ((size_t)img * a.h + yy) * a.w + xx;
                    xr[j] = load8(a.x + src * a.ldx + a.xoff + c0 + ch8 * 8);
                }
            }
        }
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int i = threadIdx.x + j * kConvThreads;
            if (i < WCHUNKS) {
                const int ch8 = i & 3, t = (i >> 2) % 9, n = (i >> 2) / 9;
                wr[j] = load8(a.wt + ((size_t)(n0 + n) * 9 + t) * a.cin + c0 + ch8 * 8);
            }
        }
    };
    auto stash = [&]() {
#pragma unroll
        for (int j = 0; j < XPT; ++j) {
            const int i = threadIdx.x + j * kConvThreads;
            if (i < CHUNKS) {
                const int ch8 = i & 3, px = (i >> 2) % TW, rr = (i >> 2) / TW;
                *(bf16x8*)&tile[(rr * TW + px) * kConvPix + ch8 * 8] = xr[j];
            }
        }
#pragma unroll
        for (int j = 0; j < WPT; ++j) {
            const int i = threadIdx.x + j * kConvThreads;
            if (i < WCHUNKS) {
                const int ch8 = i & 3, t = (i >> 2) % 9, n = (i >> 2) / 9;
                *(bf16x8*)&wtile[n * WS + t * 32 + ch8 * 8] = wr[j];
            }
        }
    };

    if (PF) fetch(0);
    for (int c0 = 0; c0 < a.cin; c0 += 32) {
        if (!PF) fetch(c0);
        stash();
        __syncthreads();
        if (PF && c0 + 32 < a.cin) fetch(c0 + 32);
        if (active) {
#pragma unroll
            for (int t = 0; t < 9; ++t) {
                const int dy = t / 3 - 1, dx = t % 3 - 1;
                bf16x8 A[MB], Bm[NB];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
                    A[mb] = *(const bf16x8*)&tile[((wv + 1 + dy) * TW + mb * 16 + l16 + 1 + dx) * kConvPix + lq * 8];
#pragma unroll
                for (int nb = 0; nb < NB; ++nb)
                    Bm[nb] = *(const bf16x8*)&wtile[(nb * 16 + l16) * WS + t * 32 + lq * 8];
#pragma unroll
                for (int mb = 0; mb < MB; ++mb)
#pragma unroll
                    for (int nb = 0; nb < NB; ++nb) acc[mb][nb] = mfma(A[mb], Bm[nb], acc[mb][nb]);
            }
        }
        __syncthreads();
    }
    if (!active) return;
#pragma unroll
    for (int mb = 0; mb < MB; ++mb)
#pragma unroll
        for (int nb = 0; nb < NB; ++nb) {
            const int n = n0 + nb * 16 + l16;
            const float bn = a.bias ? a.bias[n] : 0.0f;
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int xx = x0 + mb * 16 + lq * 4 + i;
                const size_t p = ((size_t)img * a.h + y) * a.w + xx;
                float v = acc[mb][nb][i] + bn;
                if (a.relu) v = v > 0.0f ? v : 0.0f;
                if (OUT_F32) {
                    float* o = a.yf + p * a.ldy + a.yoff + n;
                    *o = a.accumulate ? *o + v : v;
                } else {
                    a.yb[p * a.ldy + a.yoff + n] = (__bf16)v;
                }
            }
        }
}

// ------------------------------------------------------------------ weight gradient
// Partial dW over a pixel range: part[s][n][t][c] = sum_{p in split s} dz[p][n] X[p + off_t][c]
// (GEMM M = output channels, N = input channels, K = pixels, one per tap).
// The pixels are cut into units: a column strip of kWgSeg = 32 pixels of one
// image (widths are multiples of 32) over kWgUnitRows consecutive rows.  A
// workgroup takes 32 output x 32 input channels and split s; it holds
// kWgGroups groups of three waves, and group g walks units s G + g,
// (s + nsplit) G + g, ... row by row.  Wave r of a group sums the three taps
// of tap row dy = r - 1.  Per row y the group stages in LDS, transposed so
// that pixels are contiguous (the MFMA K order), dz of the row segment and X
// of row y + 1 (pixels x0 - 1 .. x0 + 32, zero outside the image); rows y - 1
// and y are still there from the two rows before (a ring of three rows; a
// unit's first row stages all three).  Chunks of 8 channels of one pixel come
// in as 16-byte loads, a pixel pair per thread, and go out as 32-bit pixel
// pairs per channel; each group of 8 channel rows is shifted by 8 banks, so
// the stores of 32 lanes hit distinct banks while the fragment reads stay
// 16-byte aligned.  The rows two steps ahead are fetched into registers while
// a row is multiplied.  Per tap row one aligned 16-byte read and the next 4
// bytes give the B fragments of its three taps (shifted by whole BF16
// elements).  At the end the groups' sums are added in group order in LDS,
// so the partials depend only on the split count.
constexpr int kWgSeg = 32;              // pixels per row segment
constexpr int kWgUnitRows = 16;         // rows per unit
constexpr int kWgGroups = 4;
constexpr int kWgThreads = kWgGroups * 3 * 64;
constexpr int kWgPitch = 40;            // LDS elements per transposed row: 34 pixels + padding (80-byte rows)
constexpr int kWgRows = 32 * kWgPitch + 4 * 16;   // 32 channel rows, four groups shifted by 16 elements
constexpr int kWgRed = 9 * 32 + 4;      // row of the final reduction (output channel): 9 taps x 32, padded
struct WgStage {
    __bf16 x[3 * kWgRows];              // ring of three X rows: [slot][input channel][pixel x0 - 1 + i]
    __bf16 dz[kWgRows];                 // [output channel][pixel x0 + i]
};
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// offset of channel row c in a staged array
__device__ __forceinline__ int wg_row(int c) { return c * kWgPitch + (c >> 3) * 16; }

__device__ __forceinline__ unsigned pack2(__bf16 lo, __bf16 hi)
{
    return (unsigned)__builtin_bit_cast(unsigned short, lo) | ((unsigned)__builtin_bit_cast(unsigned short, hi) << 16);
}

// One thread's share of staging a row: task 0..63 a dz pixel pair and channel
// group, 64..131 an X pixel pair and channel group of one input row.
struct WgChunk {
    bf16x8 u, v;
};

__global__ __launch_bounds__(kWgThreads) void conv3x3_wgrad_kernel(WgradArgs a)
{
    static_assert(sizeof(WgStage) * kWgGroups >= 32 * kWgRed * sizeof(float), "reduction area");
    __shared__ __attribute__((aligned(16))) WgStage stage[kWgGroups];
    const int grp = threadIdx.x / 192, gt = threadIdx.x % 192;   // group, thread within the group
    const int r = gt >> 6, lane = threadIdx.x & 63, l16 = lane & 15, lq = lane >> 4;
    const int ntile = a.cout / 32, ctile = a.cin / 32;
    int b = xcd_block(blockIdx.x, gridDim.x);   // the input-channel tiles of one (nt, split) on one XCD
    const int ct = b % ctile; b /= ctile;
    const int nt = b % ntile;
    const int s = b / ntile;
    const int n0 = nt * 32, c0 = ct * 32;
    const int strips = a.w / kWgSeg, ychunks = (a.h + kWgUnitRows - 1) / kWgUnitRows;
    const int units = a.n * strips * ychunks;
    const int ustride = a.nsplit * kWgGroups;
    const int niter = (units + ustride - 1) / ustride;   // units per group, the same for every group
    WgStage& L = stage[grp];

    f32x4 acc[3][2][2];
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[d][i][j] = f32x4{0.f, 0.f, 0.f, 0.f};

    // task of this thread: dz (pair, channel group) or X (pair, channel group)
    const bool tdz = gt < 64, tx = gt >= 64 && gt < 64 + 68;
    const int tpair = tdz ? gt >> 2 : (gt - 64) >> 2, tcg = gt & 3;
    // fetch: the chunks of row segment (img, x0, y): dz row y (if ydz) and X row yx
    auto fetch = [&](WgChunk& k, int img, int x0, int y, int yx, bool ok) {
        k.u = zero8();
        k.v = zero8();
        if (!ok) return;
        if (tdz) {
            const int64_t p = ((int64_t)img * a.h + y) * a.w + x0 + 2 * tpair;
            k.u = load8(a.dz + p * a.cout + n0 + tcg * 8);
            k.v = load8(a.dz + (p + 1) * a.cout + n0 + tcg * 8);
        } else if (tx && yx >= 0 && yx < a.h) {
            const int xa = x0 - 1 + 2 * tpair;                   // pixels xa, xa + 1 (xa <= w - 1)
            auto pix = [&](int xx) {
                return a.up ? ((int64_t)img * (a.h >> 1) + (yx >> 1)) * (a.w >> 1) + (xx >> 1)
                            : ((int64_t)img * a.h + yx) * a.w + xx;
            };
            const __bf16* src = a.x + a.xoff + c0 + tcg * 8;
            if (xa >= 0) k.u = load8(src + pix(xa) * a.ldx);
            if (xa + 1 < a.w) k.v = load8(src + pix(xa + 1) * a.ldx);
        }
    };
    // stash: dz into its slot, X row into ring slot `slot`
    auto stash = [&](const WgChunk& k, int slot) {
        if (tdz) {
#pragma unroll
            for (int e = 0; e < 8; ++e) *(unsigned*)&L.dz[wg_row(tcg * 8 + e) + 2 * tpair] = pack2(k.u[e], k.v[e]);
        } else if (tx) {
#pragma unroll
            for (int e = 0; e < 8; ++e)
                *(unsigned*)&L.x[slot * kWgRows + wg_row(tcg * 8 + e) + 2 * tpair] = pack2(k.u[e], k.v[e]);
        }
    };

    for (int it = 0; it < niter; ++it) {
        const int u = (it * a.nsplit + s) * kWgGroups + grp;
        const bool uok = u < units;
        int uu = uok ? u : 0;
        const int yc = uu % ychunks; uu /= ychunks;
        const int xs = uu % strips;
        const int img = uu / strips;
        const int x0 = xs * kWgSeg, y0 = yc * kWgUnitRows;
        const int y1 = min(a.h, y0 + kWgUnitRows);
        // the unit's first rows: X rows y0 - 1 and y0 into their ring slots
        {
            WgChunk k0, k1;
            fetch(k0, img, x0, y0, y0 - 1, uok);
            fetch(k1, img, x0, y0, y0, uok);
            __syncthreads();                // the previous unit's last reads are done
            if (!tdz) {
                stash(k0, (y0 + 2) % 3);
                stash(k1, y0 % 3);
            }
        }
        // rows y0 .. y0 + kWgUnitRows - 1 (rows past y1 do nothing but keep
        // the barriers of all groups in step); two rows fetched ahead
        WgChunk pf[2];
        fetch(pf[0], img, x0, y0, y0 + 1, uok && y0 < y1);
        fetch(pf[1], img, x0, y0 + 1, y0 + 2, uok && y0 + 1 < y1);
#pragma unroll 2
        for (int j = 0; j < kWgUnitRows; ++j) {
            const int y = y0 + j;
            const bool rok = uok && y < y1;
            __syncthreads();                // the reads of the row before are done
            stash(pf[j & 1], (y + 1) % 3);
            __syncthreads();
            fetch(pf[j & 1], img, x0, y + 2, y + 3, uok && y + 2 < y1);
            if (rok) {
                bf16x8 A[2];
#pragma unroll
                for (int mb = 0; mb < 2; ++mb) A[mb] = *(const bf16x8*)&L.dz[wg_row(mb * 16 + l16) + lq * 8];
                const int slot = (y + r + 2) % 3;            // X row y + r - 1
                bf16x8 Bm[3][2];                             // [dx + 1][nb]
#pragma unroll
                for (int nb = 0; nb < 2; ++nb) {
                    const __bf16* row = &L.x[slot * kWgRows + wg_row(nb * 16 + l16) + lq * 8];
                    const u32x4 w0 = *(const u32x4*)row;      // pixels x0 - 1 + 8 lq .. + 7: tap dx = -1
                    const unsigned w1 = *(const unsigned*)(row + 8);
                    const u32x4 m0 = {__builtin_amdgcn_alignbit(w0[1], w0[0], 16), __builtin_amdgcn_alignbit(w0[2], w0[1], 16),
                                      __builtin_amdgcn_alignbit(w0[3], w0[2], 16), __builtin_amdgcn_alignbit(w1, w0[3], 16)};
                    const u32x4 p1 = {w0[1], w0[2], w0[3], w1};
                    Bm[0][nb] = __builtin_bit_cast(bf16x8, w0);
                    Bm[1][nb] = __builtin_bit_cast(bf16x8, m0);
                    Bm[2][nb] = __builtin_bit_cast(bf16x8, p1);
                }
#pragma unroll
                for (int d = 0; d < 3; ++d)
#pragma unroll
                    for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                        for (int nb = 0; nb < 2; ++nb) acc[d][mb][nb] = mfma(A[mb], Bm[d][nb], acc[d][mb][nb]);
            }
        }
    }
    // the groups' sums, added in group order: red[n][t][c] (rows of kWgRed)
    float* red = (float*)stage;
    for (int g = 0; g < kWgGroups; ++g) {
        __syncthreads();
        if (grp == g) {
#pragma unroll
            for (int d = 0; d < 3; ++d)
#pragma unroll
                for (int mb = 0; mb < 2; ++mb)
#pragma unroll
                    for (int nb = 0; nb < 2; ++nb)
#pragma unroll
                        for (int i = 0; i < 4; ++i) {
                            float& o = red[(mb * 16 + lq * 4 + i) * kWgRed + (3 * r + d) * 32 + nb * 16 + l16];
                            o = g == 0 ? acc[d][mb][nb][i] : o + acc[d][mb][nb][i];
                        }
        }
    }
    __syncthreads();
    float* out = a.part + (size_t)s * a.cout * 9 * a.cin;
    for (int i = threadIdx.x; i < 32 * 9 * 32; i += kWgThreads) {
        const int c = i & 31, t = (i >> 5) % 9, n = i / (32 * 9);
        out[((size_t)(n0 + n) * 9 + t) * a.cin + c0 + c] = red[n * kWgRed + t * 32 + c];
    }
}

// Column sums in a fixed order: out[y][j] = sum over rows i of chunk y
// (rows y chunk .. min((y+1) chunk, nrows) - 1) of a[i ld + j], j < ncols.
// A block covers kColSumCols consecutive columns (fewer when ncols is
// smaller) with the rest of its 256 threads as row lanes: lane l sums rows
// l, l + lanes, ... of the chunk, then lane 0 adds the lanes' sums in lane
// order.  Serves the split-K weight gradients and the bias gradients.
constexpr int kColSumCols = 32;
__device__ __forceinline__ void col_sum_block(const float* __restrict__ a, int64_t nrows, int64_t ncols, int64_t ld,
                                              int64_t chunk, float* __restrict__ out, int64_t bx, int64_t by)
{
    __shared__ float red[256];
    const int cw = (int)min<int64_t>(ncols, kColSumCols);
    const int lanes = 256 / cw;
    const int t = threadIdx.x, jl = t % cw, rl = t / cw;
    const int64_t j = bx * cw + jl;
    const int64_t r0 = by * chunk, r1 = min<int64_t>(r0 + chunk, nrows);
    const bool act = rl < lanes && j < ncols;
    float s = 0.0f;
    if (act) {
        // 32 rows' loads in flight at once, added in row order
        int64_t i = r0 + rl;
        for (; i + 31 * lanes < r1; i += 32 * lanes) {
            float v[32];
#pragma unroll
            for (int u = 0; u < 32; ++u) v[u] = a[(i + u * lanes) * ld + j];
#pragma unroll
            for (int u = 0; u < 32; ++u) s += v[u];
        }
        for (; i < r1; i += lanes) s += a[i * ld + j];
    }
    red[t] = s;
    __syncthreads();
    if (act && rl == 0) {
        for (int k = 1; k < lanes; ++k) s += red[t + k * cw];
        out[by * ncols + j] = s;
    }
}

__global__ __launch_bounds__(256) void col_sum_kernel(const float* __restrict__ a, int64_t nrows, int64_t ncols,
                                                      int64_t ld, int64_t chunk, float* __restrict__ out)
{
    col_sum_block(a, nrows, ncols, ld, chunk, out, blockIdx.x, blockIdx.y);
}

// The same sums for arrays of at least kColSumCols columns and few rows, one
// thread per column (256 columns per block): the thread forms the sums of
// the 256 / kColSumCols = 8 lanes of col_sum_block itself (rows l, l + 8,
// ... in order, from 0.0f) and adds them in lane order, so every column gets
// the bits col_sum_block gives it.
constexpr int kColSumLanes = 256 / kColSumCols;
constexpr int kColSumFewRows = 16;
__device__ __forceinline__ void col_sum_cols_block(const float* __restrict__ a, int64_t nrows, int64_t ncols,
                                                   float* __restrict__ out, int64_t bx)
{
    const int64_t j = bx * 256 + threadIdx.x;
    if (j >= ncols) return;
    float lane[kColSumLanes];
#pragma unroll
    for (int l = 0; l < kColSumLanes; ++l) lane[l] = 0.0f;
#pragma unroll
    for (int i = 0; i < kColSumFewRows; ++i)
        if (i < nrows) lane[i % kColSumLanes] += a[i * ncols + j];
    float s = lane[0];
#pragma unroll
    for (int l = 1; l < kColSumLanes; ++l) s += lane[l];
    out[j] = s;
}

// Two column sums in one launch (each over all its rows, one chunk): blocks
// below nbx1 take the first array (one thread per column when cols1 is set),
// the rest the second; every column is summed exactly as col_sum_kernel sums it.
__global__ __launch_bounds__(256) void col_sum2_kernel(const float* __restrict__ a, int64_t nrows, int64_t ncols,
                                                       float* __restrict__ out, int64_t nbx1, int cols1,
                                                       const float* __restrict__ a2, int64_t nrows2,
                                                       int64_t ncols2, float* __restrict__ out2)
{
    if ((int64_t)blockIdx.x < nbx1) {
        if (cols1) col_sum_cols_block(a, nrows, ncols, out, blockIdx.x);
        else col_sum_block(a, nrows, ncols, ncols, nrows, out, blockIdx.x, 0);
    } else {
        col_sum_block(a2, nrows2, ncols2, ncols2, nrows2, out2, (int64_t)blockIdx.x - nbx1, 0);
    }
}

// ------------------------------------------------------------------ elementwise
// dz (BF16, contiguous [p][c]) = dy (FP32, stride ldd at doff) where the
// activation y (BF16, stride ldy at yoff) > 0, and the FP32 channel sums of
// dz over the pixels this block visits (partials of the bias gradient):
// part[blockIdx.x][c].  Thread t takes channel group t % G (8 channels;
// G = c / 8 <= 256) of pixel slot t / G; the block walks pixel groups
// blockIdx.x, blockIdx.x + gridDim.x, ... of `slots` = 256 / G pixels.  Each
// thread sums its pixels in that order, then the slots' sums are added in
// slot order, so the partials depend only on the grid size.  Channel counts,
// strides and offsets are multiples of 8 (16-byte BF16 and 32-byte FP32
// accesses).
constexpr int kReluThreads = 256;
__global__ __launch_bounds__(kReluThreads) void relu_mask_kernel(const float* __restrict__ dy, int ldd, int doff,
                                                                 const __bf16* __restrict__ y, int ldy, int yoff,
                                                                 int64_t npix, int c, __bf16* __restrict__ dz,
                                                                 float* __restrict__ part)
{
    __shared__ float red[kReluThreads * 8];
    const int G = c / 8, slots = kReluThreads / G;
    const int t = threadIdx.x, sl = t / G, ch = (t - sl * G) * 8;
    float sum[8] = {0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f, 0.f};
    if (sl < slots) {
        const int64_t stride = (int64_t)gridDim.x * slots;
        for (int64_t p = (int64_t)blockIdx.x * slots + sl; p < npix; p += stride) {
            const bf16x8 yv = load8(y + p * ldy + yoff + ch);
            const f32x4* d = (const f32x4*)(dy + p * ldd + doff + ch);
            const f32x4 d0 = d[0], d1 = d[1];
            bf16x8 ob;
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                const float o0 = (float)yv[e] > 0.0f ? d0[e] : 0.0f;
                const float o1 = (float)yv[e + 4] > 0.0f ? d1[e] : 0.0f;
                ob[e] = (__bf16)o0;
                ob[e + 4] = (__bf16)o1;
                sum[e] += o0;
                sum[e + 4] += o1;
            }
            *(bf16x8*)(dz + p * c + ch) = ob;
        }
    }
#pragma unroll
    for (int e = 0; e < 8; ++e) red[t * 8 + e] = sum[e];
    __syncthreads();
    if (t < G) {
        for (int k = 1; k < slots; ++k)
#pragma unroll
            for (int e = 0; e < 8; ++e) sum[e] += red[(k * G + t) * 8 + e];
#pragma unroll
        for (int e = 0; e < 8; ++e) part[(int64_t)blockIdx.x * c + ch + e] = sum[e];
    }
}

// Rotated, transposed weights for the data gradient: wr[c][t][n] = w[n][8 - t][c],
// layer blockIdx.y of the table (each layer at the same offset in w and wr).
__global__ void weight_flip_kernel(const __bf16* __restrict__ w, FlipLayers L, __bf16* __restrict__ wr)
{
    const int l = blockIdx.y;
    const int cout = L.cout[l], cin = L.cin[l];
    // i runs over the output (contiguous stores, strided loads)
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)cout * 9 * cin) return;
    const int n = (int)(i % cout);
    const int tr = (int)((i / cout) % 9);
    const int c = (int)(i / ((int64_t)cout * 9));
    wr[L.off[l] + i] = w[L.off[l] + ((int64_t)n * 9 + (8 - tr)) * cin + c];
}

// Minibatch gather: sample blockIdx.y of the index list, 16-byte vectors when
// the sample size and both bases allow it.
__global__ void gather_kernel(const float* __restrict__ src, int64_t elems, GatherIdx idx, float* __restrict__ dst,
                              int vec)
{
    const int k = blockIdx.y;
    const float* a = src + (int64_t)idx.i[k] * elems;
    float* b = dst + (int64_t)k * elems;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    if (vec) {
        const int64_t n4 = elems >> 2;
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < n4; e += stride)
            ((float4*)b)[e] = ((const float4*)a)[e];
    } else {
        for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < elems; e += stride) b[e] = a[e];
    }
}

__global__ void pool2_kernel(const __bf16* __restrict__ x, int ldx, int xoff, int n, int h, int w, int c,
                             __bf16* __restrict__ y)
{
    const int64_t i8 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 8 channels per thread
    const int ho = h / 2, wo = w / 2, c8 = c / 8;
    if (i8 >= (int64_t)n * ho * wo * c8) return;
    int64_t r = i8 / c8;
    const int ch = (int)(i8 - r * c8) * 8;
    const int xo = (int)(r % wo); r /= wo;
    const int yo = (int)(r % ho);
    const int img = (int)(r / ho);
    auto at = [&](int yy, int xx) { return load8(x + (((int64_t)img * h + yy) * w + xx) * ldx + xoff + ch); };
    const bf16x8 a = at(2 * yo, 2 * xo), b = at(2 * yo, 2 * xo + 1), cc = at(2 * yo + 1, 2 * xo),
                 d = at(2 * yo + 1, 2 * xo + 1);
    bf16x8 o;
#pragma unroll
    for (int e = 0; e < 8; ++e)
        o[e] = (__bf16)(0.25f * (((float)a[e] + (float)b[e]) + ((float)cc[e] + (float)d[e])));
    *(bf16x8*)(y + i8 * 8) = o;
}

// dx[fine] (+)= dy[coarse] / 4; dx has channel stride ldx at offset xoff
__global__ void pool2_back_kernel(const float* __restrict__ dy, int n, int h, int w, int c,
                                  float* __restrict__ dx, int ldx, int xoff, int accumulate)
{
    const int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 4 channels per thread
    const int c4 = c / 4;
    if (i4 >= (int64_t)n * h * w * c4) return;
    const int64_t r0 = i4 / c4;
    const int ch = (int)(i4 - r0 * c4) * 4;
    int64_t r = r0;
    const int xx = (int)(r % w); r /= w;
    const int yy = (int)(r % h);
    const int img = (int)(r / h);
    const f32x4 g = *(const f32x4*)(dy + (((int64_t)img * (h / 2) + yy / 2) * (w / 2) + xx / 2) * c + ch);
    f32x4* o = (f32x4*)(dx + r0 * ldx + xoff + ch);
    f32x4 v;
#pragma unroll
    for (int e = 0; e < 4; ++e) v[e] = 0.25f * g[e];
    if (accumulate) {
        const f32x4 old = *o;
#pragma unroll
        for (int e = 0; e < 4; ++e) v[e] = old[e] + v[e];
    }
    *o = v;
}

// dx[coarse] = sum of the 4 fine gradients
__global__ void up2_back_kernel(const float* __restrict__ dy, int n, int h, int w, int c, float* __restrict__ dx)
{
    const int64_t i4 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;   // 4 channels per thread
    const int c4 = c / 4;
    if (i4 >= (int64_t)n * h * w * c4) return;
    int64_t r = i4 / c4;
    const int ch = (int)(i4 - r * c4) * 4;
    const int xx = (int)(r % w); r /= w;
    const int yy = (int)(r % h);
    const int img = (int)(r / h);
    const int wf = 2 * w;
    auto at = [&](int fy, int fx) { return *(const f32x4*)(dy + (((int64_t)img * 2 * h + fy) * wf + fx) * c + ch); };
    const f32x4 a = at(2 * yy, 2 * xx), b = at(2 * yy, 2 * xx + 1), cc = at(2 * yy + 1, 2 * xx),
                d = at(2 * yy + 1, 2 * xx + 1);
    f32x4 o;
#pragma unroll
    for (int e = 0; e < 4; ++e) o[e] = (a[e] + b[e]) + (cc[e] + d[e]);
    *(f32x4*)(dx + i4 * 4) = o;
}

// ------------------------------------------------------------------ head (1x1), loss
// y[p][o] = b[o] + sum_c x[p][c] w[o][c]   (FP32 weights, FP32 output), the
// products added in channel order.  A pixel's channels are loaded once, in
// groups of up to kHeadVec 16-byte chunks with their loads in flight
// together, and serve every output.
constexpr int kHeadVec = 8;    // 64 channels per group
constexpr int kHeadOut = 3;    // outputs of the head (the net's out_ch)
__global__ void head_kernel(const __bf16* __restrict__ x, int64_t npix, int cin, const float* __restrict__ w,
                            const float* __restrict__ b, int cout, float* __restrict__ y)
{
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= npix) return;
    float s[kHeadOut];
    for (int o = 0; o < cout; ++o) s[o] = b[o];
    for (int c0 = 0; c0 < cin; c0 += 8 * kHeadVec) {   // cin: a multiple of 8
        const int nv = min(kHeadVec, (cin - c0) / 8);
        bf16x8 v[kHeadVec];
#pragma unroll
        for (int k = 0; k < kHeadVec; ++k)
            if (k < nv) v[k] = load8(x + p * cin + c0 + 8 * k);
        for (int o = 0; o < cout; ++o)
#pragma unroll
            for (int k = 0; k < kHeadVec; ++k)
                if (k < nv)
#pragma unroll
                    for (int e = 0; e < 8; ++e) s[o] = __builtin_fmaf((float)v[k][e], w[o * cin + c0 + 8 * k + e], s[o]);
    }
    for (int o = 0; o < cout; ++o) y[p * cout + o] = s[o];
}

// dx[p][c] = sum_o dy[p][o] w[o][c]
// dx[p][c] = sum over o, in order, of dy[p][o] w[o][c]: a thread takes four
// channels of one pixel (16-byte stores), a block ppb = 256 / (cin / 4) pixels.
__global__ __launch_bounds__(256) void head_back_kernel(const float* __restrict__ dy, int64_t npix, int cout,
                                                        const float* __restrict__ w, int cin, float* __restrict__ dx)
{
    const int c4n = cin >> 2, ppb = 256 / c4n;
    const int t = threadIdx.x, pl = t / c4n;
    if (pl >= ppb) return;
    const int64_t p = (int64_t)blockIdx.x * ppb + pl;
    if (p >= npix) return;
    const int c = (t - pl * c4n) * 4;
    float4 s = {0.0f, 0.0f, 0.0f, 0.0f};
    for (int o = 0; o < cout; ++o) {
        const float d = dy[p * cout + o];
        const float4 wv = *(const float4*)(w + (size_t)o * cin + c);
        s.x = __builtin_fmaf(d, wv.x, s.x);
        s.y = __builtin_fmaf(d, wv.y, s.y);
        s.z = __builtin_fmaf(d, wv.z, s.z);
        s.w = __builtin_fmaf(d, wv.w, s.w);
    }
    *(float4*)(dx + p * cin + c) = s;
}

// part[chunk][o][c] = sum over the chunk's pixels of dy[p][o] x[p][c]
__global__ void head_wgrad_partial_kernel(const float* __restrict__ dy, const __bf16* __restrict__ x, int64_t npix,
                                          int cout, int cin, int chunk, float* __restrict__ part)
{
    const int j = threadIdx.x + blockIdx.y * blockDim.x;   // o * cin + c
    if (j >= cout * cin) return;
    const int o = j / cin, c = j % cin;
    const int64_t b = (int64_t)blockIdx.x * chunk, e = min<int64_t>(b + chunk, npix);
    float s = 0.0f;
    int64_t p = b;
    // sixteen pixels' loads in flight at once, added in pixel order
    for (; p + 15 < e; p += 16) {
        float d[16], xv[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            d[u] = dy[(p + u) * cout + o];
            xv[u] = (float)x[(p + u) * cin + c];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) s = __builtin_fmaf(d[u], xv[u], s);
    }
    for (; p < e; ++p) s = __builtin_fmaf(dy[p * cout + o], (float)x[p * cin + c], s);
    part[(size_t)blockIdx.x * cout * cin + j] = s;
}

// Masked MSE: dy = 2 m (y - t) / cnt, partial sums of m (y - t)^2 in FP64 per block.
__global__ void mse_kernel(const float* __restrict__ y, const float* __restrict__ t, const float* __restrict__ mask,
                           int64_t npix, int c, double inv_cnt, float* __restrict__ dy, double* __restrict__ part)
{
    __shared__ double red[256];
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    double s = 0.0;
    if (i < npix * c) {
        const float m = mask ? mask[i / c] : 1.0f;
        const float r = (y[i] - t[i]) * m;
        dy[i] = (float)(2.0 * inv_cnt) * r;
        s = (double)r * (double)r;
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = red[0];
}

// One block of 256 threads: thread t sums part[t], part[t + 256], ..., then a
// fixed-order tree over the threads.
__global__ __launch_bounds__(256) void sum_f64_kernel(const double* __restrict__ part, int n, double scale,
                                                      double* __restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int i = threadIdx.x; i < n; i += 256) s += part[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) *out = red[0] * scale;
}

// ------------------------------------------------------------------ AdamW
// theta -= lr (mhat / (sqrt(vhat) + eps) + wd theta), FP32 masters; bf16 copies
// of conv weights refreshed through the map wmap (index into bf16 array, -1: none).
__global__ void adamw_kernel(float* __restrict__ th, const float* __restrict__ g, float* __restrict__ m,
                             float* __restrict__ v, int64_t n, float lr, float b1, float b2, float eps, float wd,
                             float c1, float c2, const int64_t* __restrict__ wmap, __bf16* __restrict__ wb)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.0f - b1) * gi;
    const float vi = b2 * v[i] + (1.0f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float mh = mi / c1, vh = vi / c2;
    const float t = th[i] - lr * (mh / (sqrtf(vh) + eps) + wd * th[i]);
    th[i] = t;
    const int64_t k = wmap[i];
    if (k >= 0) wb[k] = (__bf16)t;
}

__global__ void f32_to_bf16_kernel(const float* __restrict__ src, int64_t n, __bf16* __restrict__ dst)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (__bf16)src[i];
}

// Input features (FP32 [p][nin]) -> BF16 [p][ldc] with zero padding channels;
// one thread per 8 output channels of a pixel (ldc a multiple of 8).
__global__ void pack_input_kernel(const float* __restrict__ x, int64_t npix, int nin, int ldc, __bf16* __restrict__ y)
{
    const int64_t i8 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int c8 = ldc / 8;
    if (i8 >= npix * c8) return;
    const int64_t p = i8 / c8;
    const int c0 = (int)(i8 - p * c8) * 8;
    bf16x8 v;
#pragma unroll
    for (int e = 0; e < 8; ++e) v[e] = (__bf16)(c0 + e < nin ? x[p * nin + c0 + e] : 0.0f);
    *(bf16x8*)(y + i8 * 8) = v;
}

// ------------------------------------------------------------------ launchers
static inline unsigned blocks_for(int64_t n, int per) { return (unsigned)((n + per - 1) / per); }

// out[y][j] for nchunk row chunks of a [nrows][ld] array (see col_sum_kernel).
static void col_sum(const float* a, int64_t nrows, int64_t ncols, int64_t ld, int nchunk, float* out, hipStream_t s)
{
    const int64_t chunk = (nrows + nchunk - 1) / nchunk;
    const int cw = (int)std::min<int64_t>(ncols, kColSumCols);
    hipLaunchKernelGGL(col_sum_kernel, dim3(blocks_for(ncols, cw), (unsigned)((nrows + chunk - 1) / chunk)), dim3(256),
                       0, s, a, nrows, ncols, ld, chunk, out);
}

template <int MB, int NB, bool PF>
static void conv3x3_launch(const ConvArgs& a, hipStream_t s)
{
    const int64_t blocks = (int64_t)a.n * ((a.h + kConvRows - 1) / kConvRows) * (a.w / (16 * MB)) *
                           (a.cout / (16 * NB));
    if (a.yf) hipLaunchKernelGGL((conv3x3_lds_kernel<true, MB, NB, PF>), dim3((unsigned)blocks), dim3(kConvThreads), 0, s, a);
    else hipLaunchKernelGGL((conv3x3_lds_kernel<false, MB, NB, PF>), dim3((unsigned)blocks), dim3(kConvThreads), 0, s, a);
}

template <int MB, int NB>
static void conv3x3_launch(const ConvArgs& a, hipStream_t s)
{
    // prefetching pays where a workgroup runs several blocks; its registers
    // leave one workgroup per CU, so with one or two blocks two workgroups
    // per CU without it overlap better (measured 3 % faster forward passes
    // with the threshold at 64 input channels than at 32)
    if (a.cin > 64) conv3x3_launch<MB, NB, true>(a, s);
    else conv3x3_launch<MB, NB, false>(a, s);
}

// Output tile per wave: 64 x 64 (pixels x channels) where the layer allows,
// unless that launches fewer than 256 workgroups (the CUs of an MI355X):
// then 64 x 32, 32 x 64 or 32 x 32, the first that fills the chip (the deep,
// small levels; measured 7 % faster forward passes at 256^2, batch 8, than
// 64 x 64 there).
constexpr int64_t kConvMinBlocks = 256;
hipError_t conv3x3(const ConvArgs& a, hipStream_t s)
{
    // widths are multiples of 32 and channel counts of 32 (checked at net creation)
    bool wide = a.w % 64 == 0, deep = a.cout % 64 == 0;
    const int64_t groups = (int64_t)a.n * ((a.h + kConvRows - 1) / kConvRows);
    auto blocks = [&](bool wd, bool dp) { return groups * (a.w / (wd ? 64 : 32)) * (a.cout / (dp ? 64 : 32)); };
    if (wide && deep && blocks(true, true) < kConvMinBlocks) {
        if (blocks(true, false) >= kConvMinBlocks) deep = false;
        else if (blocks(false, true) >= kConvMinBlocks) wide = false;
        else wide = deep = false;
    } else if ((wide || deep) && blocks(wide, deep) < kConvMinBlocks) {
        wide = deep = false;
    }
    if (wide && deep) conv3x3_launch<4, 4>(a, s);
    else if (wide) conv3x3_launch<4, 2>(a, s);
    else if (deep) conv3x3_launch<2, 4>(a, s);
    else conv3x3_launch<2, 2>(a, s);
    return hipGetLastError();
}

hipError_t conv3x3_wgrad(const WgradArgs& a, float* dw, hipStream_t s)
{
    if (a.w % kWgSeg || a.cout % 32 || a.cin % 32 || a.nsplit < 1) return hipErrorInvalidValue;
    const int64_t blocks = (int64_t)(a.cout / 32) * (a.cin / 32) * a.nsplit;
    hipLaunchKernelGGL(conv3x3_wgrad_kernel, dim3((unsigned)blocks), dim3(kWgThreads), 0, s, a);
    const int64_t len = (int64_t)a.cout * 9 * a.cin;
    if (a.bpart) {
        // the split-K sums and the bias partials of the same layer, one launch
        const int cols1 = len >= kColSumCols && a.nsplit <= kColSumFewRows;
        const int64_t nb1 = cols1 ? blocks_for(len, 256) : blocks_for(len, (int)std::min<int64_t>(len, kColSumCols));
        const int64_t nb2 = blocks_for(a.cout, (int)std::min<int64_t>(a.cout, kColSumCols));
        hipLaunchKernelGGL(col_sum2_kernel, dim3((unsigned)(nb1 + nb2)), dim3(256), 0, s, a.part, (int64_t)a.nsplit, len,
                           dw, nb1, cols1, a.bpart, (int64_t)a.bparts, (int64_t)a.cout, a.db);
    } else {
        col_sum(a.part, a.nsplit, len, len, 1, dw, s);
    }
    return hipGetLastError();
}

hipError_t chan_sum(const float* g, int64_t npix, int c, int ld, float* part, int nchunk, float* dst, hipStream_t s)
{
    // part holds nchunk x c partial sums (the chunk count can come out lower)
    col_sum(g, npix, c, ld, nchunk, part, s);
    const int64_t chunk = (npix + nchunk - 1) / nchunk;
    col_sum(part, (npix + chunk - 1) / chunk, c, c, 1, dst, s);
    return hipGetLastError();
}

hipError_t relu_mask(const float* dy, int ldd, int doff, const __bf16* y, int ldy, int yoff, int64_t npix, int c,
                     __bf16* dz, float* part, int max_blocks, float* db, int* nparts, hipStream_t s)
{
    if (c % 8 || c / 8 > kReluThreads || ldd % 4 || doff % 4 || ldy % 8 || yoff % 8 || npix < 1 || max_blocks < 1)
        return hipErrorInvalidValue;
    const int slots = kReluThreads / (c / 8);
    const int nb = (int)std::min<int64_t>(max_blocks, (npix + slots - 1) / slots);
    hipLaunchKernelGGL(relu_mask_kernel, dim3(nb), dim3(kReluThreads), 0, s, dy, ldd, doff, y, ldy, yoff, npix, c, dz,
                       part);
    if (nparts) *nparts = nb;
    if (db) col_sum(part, nb, c, c, 1, db, s);
    return hipGetLastError();
}

hipError_t weight_flip_all(const __bf16* w, const FlipLayers& L, __bf16* wr, hipStream_t s)
{
    if (L.count < 1 || L.count > kFlipMaxLayers) return hipErrorInvalidValue;
    int64_t most = 0;
    for (int l = 0; l < L.count; ++l) most = std::max<int64_t>(most, (int64_t)L.cout[l] * 9 * L.cin[l]);
    hipLaunchKernelGGL(weight_flip_kernel, dim3(blocks_for(most, 256), (unsigned)L.count), dim3(256), 0, s, w, L, wr);
    return hipGetLastError();
}

hipError_t gather_samples(const float* src, int64_t elems, const GatherIdx& idx, float* dst, hipStream_t s)
{
    if (idx.count < 1 || idx.count > kGatherMax || elems < 1) return hipErrorInvalidValue;
    const int vec = (elems % 4 == 0) && ((uintptr_t)src % 16 == 0) && ((uintptr_t)dst % 16 == 0);
    const int64_t work = vec ? elems / 4 : elems;
    const unsigned bx = (unsigned)std::min<int64_t>(blocks_for(work, 256), 1024);
    hipLaunchKernelGGL(gather_kernel, dim3(bx, (unsigned)idx.count), dim3(256), 0, s, src, elems, idx, dst, vec);
    return hipGetLastError();
}

hipError_t pool2(const __bf16* x, int ldx, int xoff, int n, int h, int w, int c, __bf16* y, hipStream_t s)
{
    if (c % 8 || ldx % 8 || xoff % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool2_kernel, dim3(blocks_for((int64_t)n * (h / 2) * (w / 2) * c / 8, 256)), dim3(256), 0, s,
                       x, ldx, xoff, n, h, w, c, y);
    return hipGetLastError();
}

hipError_t pool2_back(const float* dy, int n, int h, int w, int c, float* dx, int ldx, int xoff, int accumulate,
                      hipStream_t s)
{
    if (c % 4 || ldx % 4 || xoff % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pool2_back_kernel, dim3(blocks_for((int64_t)n * h * w * c / 4, 256)), dim3(256), 0, s,
                       dy, n, h, w, c, dx, ldx, xoff, accumulate);
    return hipGetLastError();
}

hipError_t up2_back(const float* dy, int n, int h, int w, int c, float* dx, hipStream_t s)
{
    if (c % 4) return hipErrorInvalidValue;
    hipLaunchKernelGGL(up2_back_kernel, dim3(blocks_for((int64_t)n * h * w * c / 4, 256)), dim3(256), 0, s, dy, n, h, w, c, dx);
    return hipGetLastError();
}

hipError_t head(const __bf16* x, int64_t npix, int cin, const float* w, const float* b, int cout, float* y, hipStream_t s)
{
    if (cin % 8 || cout < 1 || cout > kHeadOut) return hipErrorInvalidValue;
    hipLaunchKernelGGL(head_kernel, dim3(blocks_for(npix, 256)), dim3(256), 0, s, x, npix, cin, w, b, cout, y);
    return hipGetLastError();
}

hipError_t head_back(const float* dy, const __bf16* x, int64_t npix, int cout, int cin, const float* w,
                     float* dx, float* part, int nchunk, float* dw, float* db, float* bpart, hipStream_t s)
{
    // four channels per thread, whole pixels per block (cin a multiple of 8, at most 1024)
    if (cin % 8 || cin > 1024 || (uintptr_t)w % 16 || (uintptr_t)dx % 16) return hipErrorInvalidValue;
    const int ppb = 256 / (cin / 4);
    hipLaunchKernelGGL(head_back_kernel, dim3(blocks_for(npix, ppb)), dim3(256), 0, s, dy, npix, cout, w, cin, dx);
    const int chunk = (int)((npix + nchunk - 1) / nchunk);
    hipLaunchKernelGGL(head_wgrad_partial_kernel, dim3(nchunk, (cout * cin + 255) / 256), dim3(256), 0, s,
                       dy, x, npix, cout, cin, chunk, part);
    col_sum(part, nchunk, (int64_t)cout * cin, (int64_t)cout * cin, 1, dw, s);
    return chan_sum(dy, npix, cout, cout, bpart, nchunk, db, s);
}

hipError_t mse(const float* y, const float* t, const float* mask, int64_t npix, int c, double inv_cnt, float* dy,
               double* part, double* out, hipStream_t s)
{
    const unsigned nb = blocks_for(npix * c, 256);
    hipLaunchKernelGGL(mse_kernel, dim3(nb), dim3(256), 0, s, y, t, mask, npix, c, inv_cnt, dy, part);
    hipLaunchKernelGGL(sum_f64_kernel, dim3(1), dim3(256), 0, s, part, (int)nb, inv_cnt, out);
    return hipGetLastError();
}

hipError_t adamw(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 float wd, float c1, float c2, const int64_t* wmap, __bf16* wb, hipStream_t s)
{
    hipLaunchKernelGGL(adamw_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, th, g, m, v, n, lr, b1, b2, eps, wd,
                       c1, c2, wmap, wb);
    return hipGetLastError();
}

hipError_t f32_to_bf16(const float* src, int64_t n, __bf16* dst, hipStream_t s)
{
    hipLaunchKernelGGL(f32_to_bf16_kernel, dim3(blocks_for(n, 256)), dim3(256), 0, s, src, n, dst);
    return hipGetLastError();
}

hipError_t pack_input(const float* x, int64_t npix, int nin, int ldc, __bf16* y, hipStream_t s)
{
    if (ldc % 8) return hipErrorInvalidValue;
    hipLaunchKernelGGL(pack_input_kernel, dim3(blocks_for(npix * ldc / 8, 256)), dim3(256), 0, s, x, npix, nin, ldc, y);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace mlb

namespace mlb {
namespace nn {

__global__ void features_kernel(const float* __restrict__ H, int nx, int ny, int ld, float m0, float s0,
                                float f1, float f2, float f3, float f4, float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny) return;
    const int x = (int)(i % nx), y = (int)(i / nx);
    float* o = out + i * kNetFeatures;
    o[0] = (H[(size_t)y * ld + x] - m0) / s0;
    o[1] = f1; o[2] = f2; o[3] = f3; o[4] = f4;
    o[5] = nx > 1 ? 2.0f * (float)x / (float)(nx - 1) - 1.0f : 0.0f;   // node position in [-1, 1]
    o[6] = ny > 1 ? 2.0f * (float)y / (float)(ny - 1) - 1.0f : 0.0f;
    o[7] = 1.0f;
}

// Per-basin channels 1..4 are uniform: computed here in FP64 and rounded once.
hipError_t features(const float* H, int nx, int ny, int ld, const float* mean, const float* stdv, double tx,
                    double ty, double cb, float tau_ref, float* out, hipStream_t s)
{
    const double mag = std::sqrt(tx * tx + ty * ty);
    double f1, f2;
    if (tau_ref > 0.0f) {
        f1 = mag > 0.0 ? tx / mag : 0.0;
        f2 = mag > 0.0 ? ty / mag : 0.0;
    } else {
        f1 = (tx - mean[1]) / stdv[1];
        f2 = (ty - mean[2]) / stdv[2];
    }
    const double f3 = (mag - mean[3]) / stdv[3], f4 = (cb - mean[4]) / stdv[4];
    hipLaunchKernelGGL(features_kernel, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, s, H, nx, ny, ld,
                       mean[0], stdv[0], (float)f1, (float)f2, (float)f3, (float)f4, out);
    return hipGetLastError();
}

__global__ void targets_kernel(const float* __restrict__ eta, const float* __restrict__ qx,
                               const float* __restrict__ qy, int nx, int ny, int ld, float ie, float iq,
                               float* __restrict__ out)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny) return;
    const size_t o = (size_t)(i / nx) * ld + (i % nx);
    out[i * 3 + 0] = eta[o] * ie;
    out[i * 3 + 1] = qx[o] * iq;
    out[i * 3 + 2] = qy[o] * iq;
}

hipError_t targets(const float* eta, const float* qx, const float* qy, int nx, int ny, int ld, float inv_eta,
                   float inv_q, float* out, hipStream_t s)
{
    hipLaunchKernelGGL(targets_kernel, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, s, eta, qx, qy, nx,
                       ny, ld, inv_eta, inv_q, out);
    return hipGetLastError();
}

// Sum of s_eta * y0 over all nodes in FP64: one block, fixed order.
__global__ void guess_mean_kernel(const float* __restrict__ y, int64_t n, float s_eta, double* __restrict__ out)
{
    __shared__ double red[256];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) s += (double)(s_eta * y[i * 3]);
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = red[0] / (double)n;
}

__global__ void guess_write_kernel(const float* __restrict__ y, int nx, int ny, int ld, float s_eta, float s_q,
                                   int w0, int w1, int w2, int w3, const double* __restrict__ mean,
                                   float* eta0, float* qx0, float* qy0, float* eta1, float* qx1, float* qy1)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny) return;
    const int x = (int)(i % nx), yy = (int)(i / nx);
    const bool wall = (w0 && x == 0) || (w1 && x == nx - 1) || (w2 && yy == 0) || (w3 && yy == ny - 1);
    const float e = (float)((double)(s_eta * y[i * 3]) - mean[0]);
    const float a = wall ? 0.0f : s_q * y[i * 3 + 1];
    const float b = wall ? 0.0f : s_q * y[i * 3 + 2];
    const size_t o = (size_t)yy * ld + x;
    eta0[o] = e; qx0[o] = a; qy0[o] = b;
    eta1[o] = e; qx1[o] = a; qy1[o] = b;
}

// ys = y smoothed by the 3x3 binomial filter (1 2 1)^T (1 2 1) / 16, edges
// clamped: it removes the grid-scale (checkerboard) content of a guess, which
// the step damps only slowly and which in FP32 can settle into a cycle whose
// per-step change keeps the residual above a tight tolerance.
__global__ void guess_smooth_kernel(const float* __restrict__ y, int nx, int ny, float* __restrict__ ys)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (int64_t)nx * ny) return;
    const int x = (int)(i % nx), yy = (int)(i / nx);
    const int xm = x > 0 ? x - 1 : 0, xp = x < nx - 1 ? x + 1 : nx - 1;
    const int ym = yy > 0 ? yy - 1 : 0, yp = yy < ny - 1 ? yy + 1 : ny - 1;
    for (int c = 0; c < 3; ++c) {
        auto at = [&](int a, int b) { return y[((int64_t)b * nx + a) * 3 + c]; };
        const float r0 = (at(xm, ym) + 2.0f * at(x, ym)) + at(xp, ym);
        const float r1 = (at(xm, yy) + 2.0f * at(x, yy)) + at(xp, yy);
        const float r2 = (at(xm, yp) + 2.0f * at(x, yp)) + at(xp, yp);
        ys[i * 3 + c] = 0.0625f * ((r0 + 2.0f * r1) + r2);
    }
}

hipError_t guess_to_state(const float* y, int nx, int ny, int ld, float s_eta, float s_q, const int* wall4,
                          double* scratch, float* ys, float* eta0, float* qx0, float* qy0, float* eta1, float* qx1,
                          float* qy1, hipStream_t s)
{
    hipLaunchKernelGGL(guess_smooth_kernel, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, s, y, nx, ny, ys);
    y = ys;
    hipLaunchKernelGGL(guess_mean_kernel, dim3(1), dim3(256), 0, s, y, (int64_t)nx * ny, s_eta, scratch);
    hipLaunchKernelGGL(guess_write_kernel, dim3(blocks_for((int64_t)nx * ny, 256)), dim3(256), 0, s, y, nx, ny,
                       ld, s_eta, s_q, wall4[0], wall4[1], wall4[2], wall4[3], scratch, eta0, qx0, qy0, eta1, qx1,
                       qy1);
    return hipGetLastError();
}

__global__ void sample_sums_kernel(const float* __restrict__ a, int64_t len, double* __restrict__ out)
{
    __shared__ double red[256];
    const float* p = a + (int64_t)blockIdx.x * len;
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < len; i += 256) s += (double)p[i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int k = 128; k >= 1; k >>= 1) {
        if ((int)threadIdx.x < k) red[threadIdx.x] += red[threadIdx.x + k];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[blockIdx.x] = red[0];
}

hipError_t sample_sums(const float* a, int n, int64_t len, double* out, hipStream_t s)
{
    hipLaunchKernelGGL(sample_sums_kernel, dim3(n), dim3(256), 0, s, a, len, out);
    return hipGetLastError();
}

__global__ void add_f64_kernel(const double* __restrict__ src, double* __restrict__ dst)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) *dst += *src;
}

hipError_t add_f64(const double* src, double* dst, hipStream_t s)
{
    hipLaunchKernelGGL(add_f64_kernel, dim3(1), dim3(64), 0, s, src, dst);
    return hipGetLastError();
}

constexpr int kNormBlocks = 256;

// part[k][block][2]: partial sums of (a - b)^2 and b^2 over a grid-stride range.
__global__ void diff_norms_partial_kernel(const float* __restrict__ a, const float* __restrict__ b, int64_t n,
                                          int64_t stride, double* __restrict__ part)
{
    __shared__ double r0[256], r1[256];
    const int k = blockIdx.y;
    const float* pa = a + k * stride;
    const float* pb = b + k * stride;
    double s0 = 0.0, s1 = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
        const double d = (double)pa[i] - (double)pb[i];
        s0 += d * d;
        s1 += (double)pb[i] * (double)pb[i];
    }
    r0[threadIdx.x] = s0;
    r1[threadIdx.x] = s1;
    __syncthreads();
    for (int m = 128; m >= 1; m >>= 1) {
        if ((int)threadIdx.x < m) {
            r0[threadIdx.x] += r0[threadIdx.x + m];
            r1[threadIdx.x] += r1[threadIdx.x + m];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[((size_t)k * gridDim.x + blockIdx.x) * 2 + 0] = r0[0];
        part[((size_t)k * gridDim.x + blockIdx.x) * 2 + 1] = r1[0];
    }
}

__global__ void diff_norms_final_kernel(const double* __restrict__ part, int nblk, double* __restrict__ out)
{
    const int j = threadIdx.x;   // 0..5: field k = j / 2, sum j % 2
    if (j >= 6) return;
    double s = 0.0;
    for (int i = 0; i < nblk; ++i) s += part[((size_t)(j / 2) * nblk + i) * 2 + (j % 2)];
    out[j] = s;
}

hipError_t diff_norms3(const float* a, const float* b, int64_t n, int64_t stride, double* part, double* out,
                       hipStream_t s)
{
    hipLaunchKernelGGL(diff_norms_partial_kernel, dim3(kNormBlocks, 3), dim3(256), 0, s, a, b, n, stride, part);
    hipLaunchKernelGGL(diff_norms_final_kernel, dim3(1), dim3(64), 0, s, part, kNormBlocks, out);
    return hipGetLastError();
}

}  // namespace nn
}  // namespace mlb
