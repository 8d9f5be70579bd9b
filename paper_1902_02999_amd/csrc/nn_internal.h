// Internal interface of the warm-start network kernels (nn_kernels.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlb {
namespace nn {

constexpr int kNetFeatures = 8;   // input features per pixel (MLB_NET_FEATURES)

// 3x3 "same" convolution, stride 1, as an implicit GEMM.  Requirements:
// w % 32 == 0, cin % 32 == 0, cout % 32 == 0, channel strides / offsets % 8 == 0.
struct ConvArgs {
    const __bf16* x;     // [n][h][w][ldx], channels xoff .. xoff + cin
    int ldx, xoff;
    int up;              // x is [n][h/2][w/2][ldx], read nearest-upsampled: pixel (y, x) is x's (y/2, x/2)
    const __bf16* wt;    // [cout][9][cin]
    const float* bias;   // [cout] or null
    __bf16* yb;          // BF16 output [n][h][w][ldy] at yoff (when yf is null)
    float* yf;           // FP32 output [n][h][w][ldy] at yoff, or null
    int ldy, yoff;
    int n, h, w, cin, cout;
    int relu;            // apply max(., 0)
    int accumulate;      // FP32 output only: add to the existing values
};

// Weight gradient with a deterministic split-K over pixels.
struct WgradArgs {
    const __bf16* dz;    // [n][h][w][cout] contiguous
    const __bf16* x;     // [n][h][w][ldx] at xoff
    int ldx, xoff;
    int up;              // x is [n][h/2][w/2][ldx], read nearest-upsampled (as ConvArgs::up)
    int n, h, w, cin, cout;
    int nsplit;
    float* part;         // [nsplit][cout][9][cin]
    const float* bpart;  // or null: [bparts][cout] bias partials, summed into db by the same final launch
    int bparts;
    float* db;
};

hipError_t conv3x3(const ConvArgs& a, hipStream_t s);
hipError_t conv3x3_wgrad(const WgradArgs& a, float* dw, hipStream_t s);
hipError_t chan_sum(const float* g, int64_t npix, int c, int ld, float* part, int nchunk, float* dst, hipStream_t s);
// dz = dy masked by y > 0 (BF16, contiguous) and db = the channel sums of dz
// (FP32, fixed order; part holds max_blocks x c partials, *nparts of them
// used).  db null: the partials are left for the caller to sum.
hipError_t relu_mask(const float* dy, int ldd, int doff, const __bf16* y, int ldy, int yoff, int64_t npix, int c,
                     __bf16* dz, float* part, int max_blocks, float* db, int* nparts, hipStream_t s);
// Rotated, transposed weights of several layers in one launch: for layer l,
// wr[off[l] + (c * 9 + 8 - t) * cout[l] + n] = w[off[l] + (n * 9 + t) * cin[l] + c].
constexpr int kFlipMaxLayers = 32;
struct FlipLayers {
    int64_t off[kFlipMaxLayers];
    int32_t cout[kFlipMaxLayers], cin[kFlipMaxLayers];
    int32_t count;
};
hipError_t weight_flip_all(const __bf16* w, const FlipLayers& L, __bf16* wr, hipStream_t s);
// dst[k] = src[idx[k]] for k < count, each sample `elems` floats (a minibatch
// gathered from a sample-major array).
constexpr int kGatherMax = 64;
struct GatherIdx {
    int32_t i[kGatherMax];
    int32_t count;
};
hipError_t gather_samples(const float* src, int64_t elems, const GatherIdx& idx, float* dst, hipStream_t s);
hipError_t pool2(const __bf16* x, int ldx, int xoff, int n, int h, int w, int c, __bf16* y, hipStream_t s);
hipError_t pool2_back(const float* dy, int n, int h, int w, int c, float* dx, int ldx, int xoff, int accumulate,
                      hipStream_t s);
hipError_t up2_back(const float* dy, int n, int h, int w, int c, float* dx, hipStream_t s);
hipError_t head(const __bf16* x, int64_t npix, int cin, const float* w, const float* b, int cout, float* y,
                hipStream_t s);
hipError_t head_back(const float* dy, const __bf16* x, int64_t npix, int cout, int cin, const float* w,
                     float* dx, float* part, int nchunk, float* dw, float* db, float* bpart, hipStream_t s);
hipError_t mse(const float* y, const float* t, const float* mask, int64_t npix, int c, double inv_cnt, float* dy,
               double* part, double* out, hipStream_t s);
hipError_t adamw(float* th, const float* g, float* m, float* v, int64_t n, float lr, float b1, float b2, float eps,
                 float wd, float c1, float c2, const int64_t* wmap, __bf16* wb, hipStream_t s);
hipError_t f32_to_bf16(const float* src, int64_t n, __bf16* dst, hipStream_t s);
hipError_t pack_input(const float* x, int64_t npix, int nin, int ldc, __bf16* y, hipStream_t s);
// Features of a basin for the net: [p][6] = ((H - m0)/s0, (tx - m1)/s1, (ty - m2)/s2,
// (cb - m3)/s3, inflow 0, wet mask 1) from the FP32 still-water depth plane (pitch ld).
hipError_t features(const float* H, int nx, int ny, int ld, const float* mean, const float* stdv, double tx,
                    double ty, double cb, float tau_ref, float* out, hipStream_t s);
// Targets [p][3] = (eta / s_eta, qx / s_q, qy / s_q) from the state planes (pitch ld).
// t = (eta, qx, qy) x (inv_eta, inv_q, inv_q)
hipError_t targets(const float* eta, const float* qx, const float* qy, int nx, int ny, int ld, float inv_eta,
                   float inv_q, float* out, hipStream_t s);
// Guess from the net output [p][3]: eta = s_eta y0 - mean, q = s_q (y1, y2), q = 0 on
// wall nodes; written into both state buffers (pitch ld).  mean over all nodes (FP64).
// Per-sample sums of a [n][len] FP32 array in FP64 (one block per sample, fixed order).
hipError_t sample_sums(const float* a, int n, int64_t len, double* out, hipStream_t s);
// dst += *src (FP64, one thread).
hipError_t add_f64(const double* src, double* dst, hipStream_t s);
// For k = 0..2: out[2k] = sum (a_k - b_k)^2, out[2k+1] = sum b_k^2 over n
// elements of the planes a + k stride, b + k stride (FP64, fixed order).
hipError_t diff_norms3(const float* a, const float* b, int64_t n, int64_t stride, double* part, double* out,
                       hipStream_t s);
hipError_t guess_to_state(const float* y, int nx, int ny, int ld, float s_eta, float s_q, const int* wall4,
                          double* scratch, float* ys, float* eta0, float* qx0, float* qy0, float* eta1, float* qx1,
                          float* qy1, hipStream_t s);

}  // namespace nn
}  // namespace mlb
