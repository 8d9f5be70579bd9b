// Host runtime of the warm-start network behind the mlb_net_* C ABI:
// parameter layout, activation / gradient buffers, forward and backward
// orchestration, AdamW, features / targets from grids, inference into a grid.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "mlb_runtime.h"
#include "nn_internal.h"

using namespace mlb;

namespace {

struct Layer {
    int cout, cin, k;         // k = 3 (conv) or 1 (head)
    int64_t woff, boff;       // offsets in the FP32 parameter vector
    int64_t wb;               // offset in the BF16 weight array (-1: head)
};

int64_t splitmix(uint64_t& s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return (int64_t)(z ^ (z >> 31));
}

double uniform01(uint64_t& s) { return ((uint64_t)splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

}  // namespace

struct mlb_net {
    mlb_ctx* ctx = nullptr;
    mlb_net_cfg cfg{};
    mlb_net_norm norm{};
    std::vector<Layer> L;
    int64_t np = 0, nwb = 0;
    float *theta = nullptr, *grad = nullptr, *m = nullptr, *v = nullptr;
    int64_t* wmap = nullptr;
    __bf16* wb = nullptr;
    __bf16* wflip = nullptr;
    int64_t step = 0;
    // activations (BF16) and gradients (FP32), index = level
    __bf16* xin = nullptr;
    std::vector<__bf16*> encin, enca, cat, deca, decb;
    __bf16* bot = nullptr;
    float* yout = nullptr;
    std::vector<float*> g_encin, g_enca, g_cat, g_upin, g_deca, g_decb;
    float* g_bot = nullptr;
    float* g_y = nullptr;
    __bf16* dz = nullptr;
    float* wpart = nullptr;
    float* cpart = nullptr;
    double* lpart = nullptr;
    double* dloss = nullptr;
    float* xstage = nullptr;   // features of one grid
    float* cold = nullptr;     // [3][h w] cold-start state (eta, qx, qy) of a warm-start run
    float* guess = nullptr;    // [3][h w] the guess
    float* fin = nullptr;      // [3][h w] the converged state
    double* npart = nullptr;   // partials of the guess-error norms
    double* nout = nullptr;    // [6] the guess-error sums
    std::vector<void*> allocs;
    size_t wpart_len = 0;

    int ch(int l) const { return cfg.base_ch << l; }
    int hh(int l) const { return cfg.height >> l; }
    int ww(int l) const { return cfg.width >> l; }
    int enc(int l, int b) const { return 2 * l + b; }
    int dec(int l, int part) const { return 2 * cfg.levels + 3 * (cfg.levels - 2 - l) + part; }
    int head() const { return (int)L.size() - 1; }
};

namespace {

template <class T>
mlb_status dalloc(mlb_net* n, T** p, size_t count)
{
    HIPCHK(hipMalloc((void**)p, count * sizeof(T) + 256));
    n->allocs.push_back(*p);
    return MLB_OK;
}

void net_free(mlb_net* n)
{
    for (void* p : n->allocs) (void)hipFree(p);
    n->allocs.clear();
}

// Blocks of the ReLU-mask kernel, each writing one partial sum of the bias
// gradient per channel (at most kBiasChunks x channels), and pixel chunks of
// the head's weight gradient (kHeadChunks x out x in, in the split-K buffer;
// its bias partials use the bias buffer).
constexpr int kBiasChunks = 1024;
constexpr int kHeadChunks = 2048;

// Pixel splits of a layer's weight gradient: about 256 workgroups (one per
// 32 x 32 channel pair and split), each of whose four groups walks at least
// one unit (a 32-pixel column strip over 16 rows).
int nsplit_for(const Layer& ly, int nb, int h, int w)
{
    const int64_t pairs = (int64_t)(ly.cout / 32) * (ly.cin / 32);
    const int64_t units = (int64_t)nb * (w / 32) * ((h + 15) / 16);
    int64_t s = std::max<int64_t>(1, 256 / std::max<int64_t>(1, pairs));
    s = std::min(s, std::max<int64_t>(1, units / 4));
    return (int)s;
}

mlb_status build(mlb_net* n)
{
    const mlb_net_cfg& c = n->cfg;
    const int Lv = c.levels;
    // layers in forward order
    int cin = c.in_ch;
    for (int l = 0; l < Lv; ++l) {
        n->L.push_back({n->ch(l), cin, 3, 0, 0, 0});
        n->L.push_back({n->ch(l), n->ch(l), 3, 0, 0, 0});
        cin = n->ch(l);
    }
    for (int l = Lv - 2; l >= 0; --l) {
        n->L.push_back({n->ch(l), n->ch(l + 1), 3, 0, 0, 0});
        n->L.push_back({n->ch(l), 2 * n->ch(l), 3, 0, 0, 0});
        n->L.push_back({n->ch(l), n->ch(l), 3, 0, 0, 0});
    }
    n->L.push_back({c.out_ch, n->ch(0), 1, 0, 0, -1});
    int64_t o = 0, ob = 0;
    for (Layer& ly : n->L) {
        ly.woff = o;
        o += (int64_t)ly.cout * ly.cin * ly.k * ly.k;
        ly.boff = o;
        o += ly.cout;
        if (ly.k == 3) {
            ly.wb = ob;
            ob += (int64_t)ly.cout * 9 * ly.cin;
        }
    }
    n->np = o;
    n->nwb = ob;
    CHK(dalloc(n, &n->theta, o));
    CHK(dalloc(n, &n->grad, o));
    CHK(dalloc(n, &n->m, o));
    CHK(dalloc(n, &n->v, o));
    CHK(dalloc(n, &n->wmap, o));
    CHK(dalloc(n, &n->wb, ob));
    CHK(dalloc(n, &n->wflip, ob));   // every conv layer's flipped weights, at its own offset
    std::vector<int64_t> wmap(o, -1);
    for (const Layer& ly : n->L)
        if (ly.k == 3)
            for (int64_t i = 0; i < (int64_t)ly.cout * 9 * ly.cin; ++i) wmap[ly.woff + i] = ly.wb + i;
    HIPCHK(hipMemcpy(n->wmap, wmap.data(), o * sizeof(int64_t), hipMemcpyHostToDevice));
    HIPCHK(hipMemset(n->m, 0, o * sizeof(float)));
    HIPCHK(hipMemset(n->v, 0, o * sizeof(float)));

    // activations for max_batch samples
    const size_t B = c.max_batch;
    auto px = [&](int l) { return B * n->hh(l) * n->ww(l); };
    CHK(dalloc(n, &n->xin, px(0) * c.in_ch));
    n->encin.assign(Lv, nullptr); n->enca.assign(Lv, nullptr); n->cat.assign(Lv, nullptr);
    n->deca.assign(Lv, nullptr); n->decb.assign(Lv, nullptr);
    n->g_encin.assign(Lv, nullptr); n->g_enca.assign(Lv, nullptr); n->g_cat.assign(Lv, nullptr);
    n->g_upin.assign(Lv, nullptr); n->g_deca.assign(Lv, nullptr); n->g_decb.assign(Lv, nullptr);
    size_t maxpc = 0;
    for (int l = 0; l < Lv; ++l) {
        const size_t p = px(l);
        if (l > 0) { CHK(dalloc(n, &n->encin[l], p * n->ch(l - 1))); CHK(dalloc(n, &n->g_encin[l], p * n->ch(l - 1))); }
        CHK(dalloc(n, &n->enca[l], p * n->ch(l)));
        CHK(dalloc(n, &n->g_enca[l], p * n->ch(l)));
        if (l < Lv - 1) {
            CHK(dalloc(n, &n->cat[l], p * 2 * n->ch(l)));
            CHK(dalloc(n, &n->g_cat[l], p * 2 * n->ch(l)));
            CHK(dalloc(n, &n->g_upin[l], p * n->ch(l + 1)));
            CHK(dalloc(n, &n->deca[l], p * n->ch(l)));
            CHK(dalloc(n, &n->g_deca[l], p * n->ch(l)));
            CHK(dalloc(n, &n->decb[l], p * n->ch(l)));
            CHK(dalloc(n, &n->g_decb[l], p * n->ch(l)));
        }
        maxpc = std::max(maxpc, p * 2 * n->ch(l));
    }
    CHK(dalloc(n, &n->bot, px(Lv - 1) * n->ch(Lv - 1)));
    CHK(dalloc(n, &n->g_bot, px(Lv - 1) * n->ch(Lv - 1)));
    CHK(dalloc(n, &n->yout, px(0) * c.out_ch));
    CHK(dalloc(n, &n->g_y, px(0) * c.out_ch));
    CHK(dalloc(n, &n->dz, maxpc));
    // split-K partials: the largest nsplit * cout * 9 * cin over layers and levels
    size_t wl = 0;
    for (int i = 0; i < (int)n->L.size() - 1; ++i) {
        const Layer& ly = n->L[i];
        const int lev = i < 2 * Lv ? i / 2 : (Lv - 2 - (i - 2 * Lv) / 3);
        wl = std::max(wl, (size_t)nsplit_for(ly, c.max_batch, n->hh(lev), n->ww(lev)) * ly.cout * 9 * ly.cin);
    }
    wl = std::max(wl, (size_t)kHeadChunks * c.out_ch * n->ch(0));
    n->wpart_len = wl;
    CHK(dalloc(n, &n->wpart, wl));
    CHK(dalloc(n, &n->cpart, std::max((size_t)kBiasChunks * n->ch(Lv - 1), (size_t)kHeadChunks * c.out_ch)));
    CHK(dalloc(n, &n->lpart, (px(0) * c.out_ch + 255) / 256 + 1));
    CHK(dalloc(n, &n->dloss, 1));
    CHK(dalloc(n, &n->xstage, (size_t)c.height * c.width * nn::kNetFeatures));
    const size_t hw = (size_t)c.height * c.width;
    CHK(dalloc(n, &n->cold, 3 * hw));
    CHK(dalloc(n, &n->guess, 3 * hw));
    CHK(dalloc(n, &n->fin, 3 * hw));
    CHK(dalloc(n, &n->npart, 3 * 256 * 2));
    CHK(dalloc(n, &n->nout, 6));
    return MLB_OK;
}

mlb_status refresh_bf16(mlb_net* n)
{
    for (const Layer& ly : n->L)
        if (ly.k == 3) HIPCHK(nn::f32_to_bf16(n->theta + ly.woff, (int64_t)ly.cout * 9 * ly.cin, n->wb + ly.wb, n->ctx->stream));
    return MLB_OK;
}

mlb_status conv_fwd(mlb_net* n, int li, const __bf16* x, int ldx, int xoff, __bf16* y, int ldy, int yoff, int lev,
                    int nb, int up = 0)
{
    const Layer& ly = n->L[li];
    nn::ConvArgs a{};
    a.x = x; a.ldx = ldx; a.xoff = xoff; a.up = up;
    a.wt = n->wb + ly.wb; a.bias = n->theta + ly.boff;
    a.yb = y; a.yf = nullptr; a.ldy = ldy; a.yoff = yoff;
    a.n = nb; a.h = n->hh(lev); a.w = n->ww(lev); a.cin = ly.cin; a.cout = ly.cout;
    a.relu = 1; a.accumulate = 0;
    HIPCHK(nn::conv3x3(a, n->ctx->stream));
    return MLB_OK;
}

// Gradients of one conv + ReLU layer: dy (FP32, stride ldd at doff) is the
// gradient of its activated output y; writes dW, db into the gradient vector
// and, when dx is given, the FP32 gradient of its input (contiguous, cin channels).
mlb_status conv_bwd(mlb_net* n, int li, const __bf16* x, int ldx, int xoff, const __bf16* y, int ldy, int yoff,
                    const float* dy, int ldd, int doff, float* dx, int lev, int nb, int up = 0)
{
    const Layer& ly = n->L[li];
    hipStream_t s = n->ctx->stream;
    const int h = n->hh(lev), w = n->ww(lev);
    const int64_t P = (int64_t)nb * h * w;
    // the bias partials are summed by the weight gradient's final launch
    int nparts = 0;
    HIPCHK(nn::relu_mask(dy, ldd, doff, y, ldy, yoff, P, ly.cout, n->dz, n->cpart, kBiasChunks, nullptr, &nparts, s));
    nn::WgradArgs g{};
    g.bpart = n->cpart; g.bparts = nparts; g.db = n->grad + ly.boff;
    g.dz = n->dz; g.x = x; g.ldx = ldx; g.xoff = xoff; g.up = up;
    g.n = nb; g.h = h; g.w = w; g.cin = ly.cin; g.cout = ly.cout;
    g.nsplit = nsplit_for(ly, nb, h, w);
    g.part = n->wpart;
    if ((size_t)g.nsplit * ly.cout * 9 * ly.cin > n->wpart_len) return fail(MLB_E_DEVICE, "split-K buffer too small");
    HIPCHK(nn::conv3x3_wgrad(g, n->grad + ly.woff, s));
    if (dx) {
        nn::ConvArgs a{};
        a.x = n->dz; a.ldx = ly.cout; a.xoff = 0;
        a.wt = n->wflip + ly.wb; a.bias = nullptr;
        a.yb = nullptr; a.yf = dx; a.ldy = ly.cin; a.yoff = 0;
        a.n = nb; a.h = h; a.w = w; a.cin = ly.cout; a.cout = ly.cin;
        a.relu = 0; a.accumulate = 0;
        HIPCHK(nn::conv3x3(a, s));
    }
    return MLB_OK;
}

mlb_status forward(mlb_net* n, const float* x, int nb)
{
    const mlb_net_cfg& c = n->cfg;
    const int Lv = c.levels;
    hipStream_t s = n->ctx->stream;
    const int64_t P0 = (int64_t)nb * c.height * c.width;
    HIPCHK(nn::pack_input(x, P0, nn::kNetFeatures, c.in_ch, n->xin, s));
    for (int l = 0; l < Lv; ++l) {
        const __bf16* in = n->xin;
        int ldin = c.in_ch;
        if (l > 0) {
            const int cp = n->ch(l - 1);
            HIPCHK(nn::pool2(n->cat[l - 1], 2 * cp, cp, nb, n->hh(l - 1), n->ww(l - 1), cp, n->encin[l], s));
            in = n->encin[l];
            ldin = cp;
        }
        CHK(conv_fwd(n, n->enc(l, 0), in, ldin, 0, n->enca[l], n->ch(l), 0, l, nb));
        if (l < Lv - 1) CHK(conv_fwd(n, n->enc(l, 1), n->enca[l], n->ch(l), 0, n->cat[l], 2 * n->ch(l), n->ch(l), l, nb));
        else CHK(conv_fwd(n, n->enc(l, 1), n->enca[l], n->ch(l), 0, n->bot, n->ch(l), 0, l, nb));
    }
    for (int l = Lv - 2; l >= 0; --l) {
        // the upsampling conv reads level l + 1 nearest-upsampled (up = 1)
        const __bf16* src = l == Lv - 2 ? n->bot : n->decb[l + 1];
        const int cu = n->ch(l + 1);
        CHK(conv_fwd(n, n->dec(l, 0), src, cu, 0, n->cat[l], 2 * n->ch(l), 0, l, nb, 1));
        CHK(conv_fwd(n, n->dec(l, 1), n->cat[l], 2 * n->ch(l), 0, n->deca[l], n->ch(l), 0, l, nb));
        CHK(conv_fwd(n, n->dec(l, 2), n->deca[l], n->ch(l), 0, n->decb[l], n->ch(l), 0, l, nb));
    }
    const Layer& hd = n->L[n->head()];
    HIPCHK(nn::head(n->decb[0], P0, hd.cin, n->theta + hd.woff, n->theta + hd.boff, hd.cout, n->yout, s));
    return MLB_OK;
}

mlb_status backward(mlb_net* n, int nb)
{
    const mlb_net_cfg& c = n->cfg;
    const int Lv = c.levels;
    hipStream_t s = n->ctx->stream;
    const int64_t P0 = (int64_t)nb * c.height * c.width;
    // rotated, transposed weights of every conv layer for the data gradients,
    // up to kFlipMaxLayers layers per launch
    nn::FlipLayers fl{};
    for (size_t i = 0; i < n->L.size(); ++i) {
        const Layer& ly = n->L[i];
        if (ly.k == 3) {
            fl.off[fl.count] = ly.wb;
            fl.cout[fl.count] = ly.cout;
            fl.cin[fl.count] = ly.cin;
            ++fl.count;
        }
        if (fl.count == nn::kFlipMaxLayers || (i + 1 == n->L.size() && fl.count > 0)) {
            HIPCHK(nn::weight_flip_all(n->wb, fl, n->wflip, s));
            fl.count = 0;
        }
    }
    const Layer& hd = n->L[n->head()];
    HIPCHK(nn::head_back(n->g_y, n->decb[0], P0, hd.cout, hd.cin, n->theta + hd.woff, n->g_decb[0], n->wpart, kHeadChunks,
                         n->grad + hd.woff, n->grad + hd.boff, n->cpart, s));
    for (int l = 0; l <= Lv - 2; ++l) {
        const int cl = n->ch(l), cu = n->ch(l + 1);
        CHK(conv_bwd(n, n->dec(l, 2), n->deca[l], cl, 0, n->decb[l], cl, 0, n->g_decb[l], cl, 0, n->g_deca[l], l, nb));
        CHK(conv_bwd(n, n->dec(l, 1), n->cat[l], 2 * cl, 0, n->deca[l], cl, 0, n->g_deca[l], cl, 0, n->g_cat[l], l, nb));
        const __bf16* src = l == Lv - 2 ? n->bot : n->decb[l + 1];
        CHK(conv_bwd(n, n->dec(l, 0), src, cu, 0, n->cat[l], 2 * cl, 0, n->g_cat[l], 2 * cl, 0, n->g_upin[l], l, nb,
                     1));
        float* dst = l + 1 <= Lv - 2 ? n->g_decb[l + 1] : n->g_bot;
        HIPCHK(nn::up2_back(n->g_upin[l], nb, n->hh(l + 1), n->ww(l + 1), cu, dst, s));
    }
    for (int l = Lv - 1; l >= 0; --l) {
        const int cl = n->ch(l);
        const bool last = l == Lv - 1;
        const __bf16* yb = last ? n->bot : n->cat[l];
        const float* gb = last ? n->g_bot : n->g_cat[l];
        const int ld = last ? cl : 2 * cl, off = last ? 0 : cl;
        CHK(conv_bwd(n, n->enc(l, 1), n->enca[l], cl, 0, yb, ld, off, gb, ld, off, n->g_enca[l], l, nb));
        const __bf16* xin = l == 0 ? n->xin : n->encin[l];
        const int ldx = l == 0 ? c.in_ch : n->ch(l - 1);
        CHK(conv_bwd(n, n->enc(l, 0), xin, ldx, 0, n->enca[l], cl, 0, n->g_enca[l], cl, 0,
                     l == 0 ? nullptr : n->g_encin[l], l, nb));
        if (l > 0) {
            const int cp = n->ch(l - 1);
            HIPCHK(nn::pool2_back(n->g_encin[l], nb, n->hh(l - 1), n->ww(l - 1), cp, n->g_cat[l - 1], 2 * cp, cp, 1, s));
        }
    }
    return MLB_OK;
}

// Per-basin output factor f: |tau|/rho / tau_ref, or 1 without stress scaling.
double out_factor(const mlb_net* n, const mlb_grid* g)
{
    if (!(n->norm.tau_ref > 0)) return 1.0;
    return std::sqrt(g->tx * g->tx + g->ty * g->ty) / (double)n->norm.tau_ref;
}

mlb_status check_grid(const mlb_net* n, const mlb_grid* g)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    if (g->ctx != n->ctx) return fail(MLB_E_INVAL, "grid and net belong to different contexts");
    if (g->p.nx != n->cfg.width || g->p.ny != n->cfg.height) return fail(MLB_E_INVAL, "grid size differs from the net's");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    return MLB_OK;
}

}  // namespace

extern "C" {

mlb_status mlb_net_create(mlb_ctx* ctx, const mlb_net_cfg* cfg, uint64_t seed, mlb_net** out)
{
    if (!ctx || !cfg || !out) return fail(MLB_E_INVAL, "NULL argument");
    *out = nullptr;
    const mlb_net_cfg& c = *cfg;
    if (c.levels < 2 || c.base_ch < 32 || c.base_ch % 32 || c.in_ch < 6 || c.in_ch % 32 || c.out_ch != 3 ||
        c.max_batch < 1)
        return fail(MLB_E_INVAL, "net config: levels >= 2, base_ch and in_ch multiples of 32, out_ch 3");
    const int f = 1 << (c.levels - 1);
    if (c.width % (32 * f) || c.height % f || c.height < f) return fail(MLB_E_INVAL, "net config: field size");
    if ((int64_t)c.base_ch * f > 2048) return fail(MLB_E_INVAL, "net config: at most 2048 channels at the deepest level");
    HIPCHK(hipSetDevice(ctx->device));
    mlb_net* n = new (std::nothrow) mlb_net();
    if (!n) return fail(MLB_E_NOMEM, "net");
    n->ctx = ctx;
    n->cfg = c;
    for (int k = 0; k < 5; ++k) { n->norm.in_mean[k] = 0.f; n->norm.in_std[k] = 1.f; }
    n->norm.s_eta = 1.f;
    n->norm.s_q = 1.f;
    n->norm.tau_ref = 0.f;
    mlb_status st = build(n);
    if (st != MLB_OK) { net_free(n); delete n; return st; }
    // He-normal weights (Box-Muller on a splitmix stream), zero biases
    std::vector<float> th(n->np, 0.0f);
    uint64_t rs = seed ^ 0x6d6c625f6e6574ull;
    for (const Layer& ly : n->L) {
        const double sd = std::sqrt(2.0 / ((double)ly.cin * ly.k * ly.k));
        const int64_t nw = (int64_t)ly.cout * ly.cin * ly.k * ly.k;
        for (int64_t i = 0; i < nw; ++i) {
            const double u1 = std::max(uniform01(rs), 1e-300), u2 = uniform01(rs);
            th[ly.woff + i] = (float)(sd * std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2));
        }
    }
    st = mlb_net_set_params(n, th.data(), n->np);
    if (st != MLB_OK) { net_free(n); delete n; return st; }
    ctx->live++;
    *out = n;
    return MLB_OK;
}

mlb_status mlb_net_destroy(mlb_net* n)
{
    if (!n) return fail(MLB_E_INVAL, "net is NULL");
    (void)hipSetDevice(n->ctx->device);
    (void)hipStreamSynchronize(n->ctx->stream);
    net_free(n);
    n->ctx->live--;
    delete n;
    return MLB_OK;
}

mlb_status mlb_net_param_count(const mlb_net* n, int64_t* np)
{
    if (!n || !np) return fail(MLB_E_INVAL, "NULL argument");
    *np = n->np;
    return MLB_OK;
}

mlb_status mlb_net_get_params(mlb_net* n, float* host, int64_t cnt)
{
    if (!n || !host || cnt != n->np) return fail(MLB_E_INVAL, "bad arguments (count must equal the parameter count)");
    HIPCHK(hipSetDevice(n->ctx->device));
    HIPCHK(hipMemcpyAsync(host, n->theta, cnt * sizeof(float), hipMemcpyDeviceToHost, n->ctx->stream));
    HIPCHK(hipStreamSynchronize(n->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_net_set_params(mlb_net* n, const float* host, int64_t cnt)
{
    if (!n || !host || cnt != n->np) return fail(MLB_E_INVAL, "bad arguments (count must equal the parameter count)");
    HIPCHK(hipSetDevice(n->ctx->device));
    HIPCHK(hipMemcpyAsync(n->theta, host, cnt * sizeof(float), hipMemcpyHostToDevice, n->ctx->stream));
    CHK(refresh_bf16(n));
    HIPCHK(hipMemsetAsync(n->m, 0, cnt * sizeof(float), n->ctx->stream));
    HIPCHK(hipMemsetAsync(n->v, 0, cnt * sizeof(float), n->ctx->stream));
    HIPCHK(hipStreamSynchronize(n->ctx->stream));
    n->step = 0;
    return MLB_OK;
}

mlb_status mlb_net_set_norm(mlb_net* n, const mlb_net_norm* nm)
{
    if (!n || !nm) return fail(MLB_E_INVAL, "NULL argument");
    for (int k = 0; k < 5; ++k)
        if (!(nm->in_std[k] > 0)) return fail(MLB_E_INVAL, "in_std must be positive");
    if (!(nm->s_eta > 0) || !(nm->s_q > 0)) return fail(MLB_E_INVAL, "output scales must be positive");
    if (!(nm->tau_ref >= 0)) return fail(MLB_E_INVAL, "tau_ref must be >= 0");
    n->norm = *nm;
    return MLB_OK;
}

mlb_status mlb_net_get_norm(const mlb_net* n, mlb_net_norm* nm)
{
    if (!n || !nm) return fail(MLB_E_INVAL, "NULL argument");
    *nm = n->norm;
    return MLB_OK;
}

mlb_status mlb_net_forward(mlb_net* n, const float* x, int32_t nb, float* y)
{
    if (!n || !x || !y || nb < 1 || nb > n->cfg.max_batch) return fail(MLB_E_INVAL, "bad forward arguments");
    HIPCHK(hipSetDevice(n->ctx->device));
    CHK(forward(n, x, nb));
    const size_t bytes = (size_t)nb * n->cfg.height * n->cfg.width * n->cfg.out_ch * sizeof(float);
    HIPCHK(hipMemcpyAsync(y, n->yout, bytes, hipMemcpyDeviceToDevice, n->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_net_loss_grad(mlb_net* n, const float* x, const float* t, const float* mask, double mask_count,
                             int32_t nb, double* loss, float* grad_host)
{
    if (!n || !x || !t || nb < 1 || nb > n->cfg.max_batch) return fail(MLB_E_INVAL, "bad loss arguments");
    if (mask && !(mask_count > 0)) return fail(MLB_E_INVAL, "mask_count must be positive");
    HIPCHK(hipSetDevice(n->ctx->device));
    hipStream_t s = n->ctx->stream;
    CHK(forward(n, x, nb));
    const int64_t P0 = (int64_t)nb * n->cfg.height * n->cfg.width;
    const double cnt = (mask ? mask_count : (double)P0) * n->cfg.out_ch;
    HIPCHK(nn::mse(n->yout, t, mask, P0, n->cfg.out_ch, 1.0 / cnt, n->g_y, n->lpart, n->dloss, s));
    CHK(backward(n, nb));
    if (loss) {
        HIPCHK(hipMemcpyAsync(loss, n->dloss, sizeof(double), hipMemcpyDeviceToHost, s));
    }
    if (grad_host) {
        HIPCHK(hipMemcpyAsync(grad_host, n->grad, n->np * sizeof(float), hipMemcpyDeviceToHost, s));
    }
    if (loss || grad_host) HIPCHK(hipStreamSynchronize(s));
    return MLB_OK;
}

mlb_status mlb_net_adamw(mlb_net* n, const mlb_adamw_cfg* a)
{
    if (!n || !a || !(a->lr > 0) || !(a->beta1 >= 0 && a->beta1 < 1) || !(a->beta2 >= 0 && a->beta2 < 1) ||
        !(a->eps > 0) || !(a->weight_decay >= 0))
        return fail(MLB_E_INVAL, "bad AdamW settings");
    HIPCHK(hipSetDevice(n->ctx->device));
    n->step++;
    const float c1 = (float)(1.0 - std::pow((double)a->beta1, (double)n->step));
    const float c2 = (float)(1.0 - std::pow((double)a->beta2, (double)n->step));
    HIPCHK(nn::adamw(n->theta, n->grad, n->m, n->v, n->np, a->lr, a->beta1, a->beta2, a->eps, a->weight_decay, c1,
                     c2, n->wmap, n->wb, n->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_net_features(mlb_net* n, mlb_grid* g, float* x)
{
    if (!n || !x) return fail(MLB_E_INVAL, "NULL argument");
    CHK(check_grid(n, g));
    HIPCHK(hipSetDevice(n->ctx->device));
    HIPCHK(nn::features(g->H, g->p.nx, g->p.ny, g->ld, n->norm.in_mean, n->norm.in_std, g->tx, g->ty, g->cb,
                        n->norm.tau_ref, x, n->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_net_targets(mlb_net* n, mlb_grid* g, float* t)
{
    if (!n || !t) return fail(MLB_E_INVAL, "NULL argument");
    CHK(check_grid(n, g));
    HIPCHK(hipSetDevice(n->ctx->device));
    const double f = out_factor(n, g);
    HIPCHK(nn::targets(g->eta[g->cur], g->qx[g->cur], g->qy[g->cur], g->p.nx, g->p.ny, g->ld,
                       f > 0 ? (float)(1.0 / (n->norm.s_eta * f)) : 0.0f,
                       f > 0 ? (float)(1.0 / (n->norm.s_q * f)) : 0.0f, t, n->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_net_infer(mlb_net* n, mlb_grid* g)
{
    if (!n) return fail(MLB_E_INVAL, "net is NULL");
    CHK(check_grid(n, g));
    if (g->dmask) return fail(MLB_E_STATE, "the warm start covers grids without a node mask");
    if (g->etal) return fail(MLB_E_STATE, "the warm start covers grids with an FP32 surface");
    HIPCHK(hipSetDevice(n->ctx->device));
    hipStream_t s = n->ctx->stream;
    HIPCHK(nn::features(g->H, g->p.nx, g->p.ny, g->ld, n->norm.in_mean, n->norm.in_std, g->tx, g->ty, g->cb,
                        n->norm.tau_ref, n->xstage, s));
    CHK(forward(n, n->xstage, 1));
    int wall4[4];
    for (int k = 0; k < 4; ++k) wall4[k] = g->p.edge[k] == MLB_EDGE_WALL;
    const double f = out_factor(n, g);
    HIPCHK(nn::guess_to_state(n->yout, g->p.nx, g->p.ny, g->ld, (float)(n->norm.s_eta * f),
                              (float)(n->norm.s_q * f), wall4, n->dloss, n->xstage,
                              g->eta[0], g->qx[0], g->qy[0], g->eta[1], g->qx[1], g->qy[1], s));
    grid_state_changed(g);
    return MLB_OK;
}

mlb_status mlb_net_save(const mlb_net* n, const char* path)
{
    if (!n || !path) return fail(MLB_E_INVAL, "NULL argument");
    std::vector<float> th(n->np);
    CHK(mlb_net_get_params(const_cast<mlb_net*>(n), th.data(), n->np));
    FILE* f = std::fopen(path, "wb");
    if (!f) return fail(MLB_E_INVAL, std::string("cannot open ") + path);
    const char magic[8] = {'M', 'L', 'B', 'N', 'E', 'T', '2', 0};
    bool ok = std::fwrite(magic, 8, 1, f) == 1 && std::fwrite(&n->cfg, sizeof(n->cfg), 1, f) == 1 &&
              std::fwrite(&n->norm, sizeof(n->norm), 1, f) == 1 && std::fwrite(&n->np, sizeof(n->np), 1, f) == 1 &&
              std::fwrite(th.data(), sizeof(float), th.size(), f) == th.size();
    ok = (std::fclose(f) == 0) && ok;
    return ok ? MLB_OK : fail(MLB_E_INVAL, "write failed");
}

mlb_status mlb_net_load(mlb_net* n, const char* path)
{
    if (!n || !path) return fail(MLB_E_INVAL, "NULL argument");
    FILE* f = std::fopen(path, "rb");
    if (!f) return fail(MLB_E_INVAL, std::string("cannot open ") + path);
    char magic[8];
    mlb_net_cfg c{};
    mlb_net_norm nm{};
    int64_t np = 0;
    bool ok = std::fread(magic, 8, 1, f) == 1 && std::memcmp(magic, "MLBNET2", 8) == 0 &&
              std::fread(&c, sizeof(c), 1, f) == 1 && std::fread(&nm, sizeof(nm), 1, f) == 1 &&
              std::fread(&np, sizeof(np), 1, f) == 1;
    std::vector<float> th;
    if (ok && np == n->np && c.levels == n->cfg.levels && c.base_ch == n->cfg.base_ch && c.in_ch == n->cfg.in_ch) {
        th.resize(np);
        ok = std::fread(th.data(), sizeof(float), np, f) == (size_t)np;
    } else {
        ok = false;
    }
    std::fclose(f);
    if (!ok) return fail(MLB_E_INVAL, "file is not a net of this architecture");
    CHK(mlb_net_set_params(n, th.data(), np));
    return mlb_net_set_norm(n, &nm);
}

mlb_status mlb_net_train(mlb_net* n, const float* x, const float* t, const float* mask, int32_t ns,
                         const mlb_train_cfg* cfg, double* epoch_loss)
{
    if (!n || !x || !t || !cfg || ns < 1) return fail(MLB_E_INVAL, "bad training arguments");
    const mlb_train_cfg& c = *cfg;
    if (c.epochs < 1 || c.batch < 1 || c.batch > n->cfg.max_batch || !(c.lr > 0) || !(c.lr_min >= 0) ||
        c.warmup_steps < 0 || !(c.beta1 >= 0 && c.beta1 < 1) || !(c.beta2 >= 0 && c.beta2 < 1) || !(c.eps > 0) ||
        !(c.weight_decay >= 0))
        return fail(MLB_E_INVAL, "bad training settings (batch must be 1..max_batch)");
    HIPCHK(hipSetDevice(n->ctx->device));
    hipStream_t s = n->ctx->stream;
    const size_t hw = (size_t)n->cfg.height * n->cfg.width;
    const size_t sx = hw * nn::kNetFeatures, st = hw * 3;
    const int B = c.batch;
    // staging of one minibatch, per-sample mask sums, per-epoch loss sums
    float *xb = nullptr, *tb = nullptr, *mb = nullptr;
    double *msum = nullptr, *eloss = nullptr;
    struct Guard {
        std::vector<void*> p;
        ~Guard() { for (void* q : p) (void)hipFree(q); }
    } guard;
    HIPCHK(hipMalloc((void**)&xb, B * sx * sizeof(float))); guard.p.push_back(xb);
    HIPCHK(hipMalloc((void**)&tb, B * st * sizeof(float))); guard.p.push_back(tb);
    HIPCHK(hipMalloc((void**)&eloss, c.epochs * sizeof(double))); guard.p.push_back(eloss);
    HIPCHK(hipMemsetAsync(eloss, 0, c.epochs * sizeof(double), s));
    std::vector<double> hsum;
    if (mask) {
        HIPCHK(hipMalloc((void**)&mb, B * hw * sizeof(float))); guard.p.push_back(mb);
        HIPCHK(hipMalloc((void**)&msum, ns * sizeof(double))); guard.p.push_back(msum);
        HIPCHK(nn::sample_sums(mask, ns, (int64_t)hw, msum, s));
        hsum.resize(ns);
        HIPCHK(hipMemcpyAsync(hsum.data(), msum, ns * sizeof(double), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
    }
    const int per_epoch = (ns + B - 1) / B;
    const int64_t total = (int64_t)per_epoch * c.epochs;
    std::vector<int> order(ns);
    for (int i = 0; i < ns; ++i) order[i] = i;
    uint64_t rs = c.seed ^ 0x747261696e6d6c62ull;
    int64_t it = 0;
    for (int ep = 0; ep < c.epochs; ++ep) {
        for (int i = ns - 1; i > 0; --i) {   // Fisher-Yates
            const int j = (int)((uint64_t)splitmix(rs) % (uint64_t)(i + 1));
            std::swap(order[i], order[j]);
        }
        for (int b0 = 0; b0 < ns; b0 += B, ++it) {
            const int nb = std::min(B, ns - b0);
            double cnt = 0.0;
            for (int k0 = 0; k0 < nb; k0 += nn::kGatherMax) {
                nn::GatherIdx gi{};
                gi.count = std::min(nb - k0, nn::kGatherMax);
                for (int k = 0; k < gi.count; ++k) {
                    gi.i[k] = order[b0 + k0 + k];
                    if (mask) cnt += hsum[gi.i[k]];
                }
                HIPCHK(nn::gather_samples(x, sx, gi, xb + (size_t)k0 * sx, s));
                HIPCHK(nn::gather_samples(t, st, gi, tb + (size_t)k0 * st, s));
                if (mask) HIPCHK(nn::gather_samples(mask, hw, gi, mb + (size_t)k0 * hw, s));
            }
            if (mask && !(cnt > 0)) continue;   // an all-dry minibatch carries no information
            CHK(mlb_net_loss_grad(n, xb, tb, mask ? mb : nullptr, cnt, nb, nullptr, nullptr));
            HIPCHK(nn::add_f64(n->dloss, eloss + ep, s));
            double lr = c.lr;
            if (it < c.warmup_steps) {
                lr = c.lr * (double)(it + 1) / (double)c.warmup_steps;
            } else {
                const double span = (double)std::max<int64_t>(1, total - c.warmup_steps);
                const double f = (double)(it - c.warmup_steps) / span;
                lr = c.lr_min + 0.5 * (c.lr - c.lr_min) * (1.0 + std::cos(M_PI * f));
            }
            mlb_adamw_cfg a{(float)lr, c.beta1, c.beta2, c.eps, c.weight_decay};
            CHK(mlb_net_adamw(n, &a));
        }
    }
    std::vector<double> el(c.epochs);
    HIPCHK(hipMemcpyAsync(el.data(), eloss, c.epochs * sizeof(double), hipMemcpyDeviceToHost, s));
    HIPCHK(hipStreamSynchronize(s));
    if (epoch_loss)
        for (int ep = 0; ep < c.epochs; ++ep) epoch_loss[ep] = el[ep] / per_epoch;
    return MLB_OK;
}

namespace {

mlb_status save_fields(mlb_net* n, mlb_grid* g, float* dst)
{
    const size_t hw = (size_t)n->cfg.height * n->cfg.width;
    return mlb_get_state_device(g, dst, dst + hw, dst + 2 * hw, nullptr);
}

// One checked chunk of at most `steps` steps; NOTCONVERGED is not an error here.
mlb_status probe(mlb_grid* g, double tol, int64_t steps, int32_t check_every, mlb_diag_t* d, bool* converged)
{
    const mlb_status st = mlb_run_steady(g, tol, steps, check_every, d);
    *converged = st == MLB_OK;
    if (st == MLB_E_NOTCONVERGED || st == MLB_OK || st == MLB_E_NONFINITE || st == MLB_E_STALLED) return MLB_OK;
    return st;
}

}  // namespace

mlb_status mlb_warm_start_run(mlb_grid* g, mlb_net* n, double tol, int64_t max_steps, int32_t check_every,
                              mlb_warm_report* rep)
{
    if (!n || !rep) return fail(MLB_E_INVAL, "NULL argument");
    if (check_every < 1 || max_steps < 2 || !(tol >= 0)) return fail(MLB_E_INVAL, "bad tol / max_steps / check_every");
    CHK(check_grid(n, g));
    if (g->dmask) return fail(MLB_E_STATE, "the warm start covers grids without a node mask");
    if (g->etal) return fail(MLB_E_STATE, "the warm start covers grids with an FP32 surface");
    HIPCHK(hipSetDevice(n->ctx->device));
    const auto t0 = std::chrono::steady_clock::now();
    hipStream_t s = n->ctx->stream;
    *rep = mlb_warm_report{};
    const int64_t step0 = g->step;
    const size_t hw = (size_t)n->cfg.height * n->cfg.width;
    bool conv = false;
    mlb_diag_t d{};

    // 1. cold-start probe
    CHK(save_fields(n, g, n->cold));
    CHK(probe(g, tol, 1, 1, &d, &conv));
    rep->r0_cold = d.nonfinite ? INFINITY : d.residual;
    rep->steps_total = 1;
    if (conv) {   // the cold start is already steady: nothing to guess
        rep->steps = 1;
        rep->diag = d;
        for (int k = 0; k < 3; ++k) rep->guess_err[k] = NAN;
        rep->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
        return MLB_OK;
    }

    // 2. the guess and its first step
    hipEvent_t e0 = nullptr, e1 = nullptr;
    HIPCHK(hipEventCreate(&e0));
    if (hipEventCreate(&e1) != hipSuccess) { (void)hipEventDestroy(e0); return fail(MLB_E_DEVICE, "hipEventCreate"); }
    float ms = 0.f;
    mlb_status ist = MLB_OK;
    if (hipEventRecord(e0, s) != hipSuccess) ist = fail(MLB_E_DEVICE, "hipEventRecord");
    if (ist == MLB_OK) ist = mlb_net_infer(n, g);
    if (ist == MLB_OK && (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                          hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
        ist = fail(MLB_E_DEVICE, "timing the inference");
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    CHK(ist);
    rep->infer_ms = ms;
    CHK(grid_set_step(g, step0));
    CHK(save_fields(n, g, n->guess));
    CHK(probe(g, tol, 1, 1, &d, &conv));
    rep->steps_total += 1;
    rep->r0_guess = d.nonfinite ? INFINITY : d.residual;
    int reason = MLB_WARM_NONE;
    if (d.nonfinite || !std::isfinite(d.residual)) reason = MLB_WARM_NONFINITE_GUESS;
    else if (rep->r0_guess > rep->r0_cold) reason = MLB_WARM_WORSE_THAN_COLD;

    // 3. the warm run, watched for divergence
    int64_t used = 1;
    bool stalled = false;
    if (reason == MLB_WARM_NONE && !conv) {
        double first = -1.0, prev = d.residual, best = d.residual;
        int rises = 0, since = 0;
        const int stall = n->ctx->stall_checks;
        while (used < max_steps) {
            const int64_t chunk = std::min<int64_t>(check_every, max_steps - used);
            CHK(probe(g, tol, chunk, check_every, &d, &conv));
            used += chunk;
            rep->steps_total += chunk;
            if (d.nonfinite) { reason = MLB_WARM_DIVERGING; break; }
            if (conv) break;
            if (first < 0) first = d.residual;
            rises = d.residual > prev ? rises + 1 : 0;
            prev = d.residual;
            if (rises >= 3 && d.residual > first) { reason = MLB_WARM_DIVERGING; break; }
            if (d.residual < best) { best = d.residual; since = 0; }
            else if (stall > 0 && best <= kStallBand * tol && ++since >= stall) { stalled = true; break; }
        }
    }
    mlb_status result = MLB_OK;
    if (reason == MLB_WARM_NONE) {
        rep->used_guess = 1;
        rep->steps = used;
        if (stalled) result = fail(MLB_E_STALLED, "residual stalled");
        else if (!conv) result = fail(MLB_E_NOTCONVERGED, "max_steps reached");
    } else {
        // 4. fallback: the cold start again
        CHK(mlb_set_state_device(g, n->cold, n->cold + hw, n->cold + 2 * hw));
        CHK(grid_set_step(g, step0));
        result = mlb_run_steady(g, tol, max_steps, check_every, &d);
        rep->steps = g->step - step0;
        rep->steps_total += rep->steps;
        conv = result == MLB_OK;
    }
    rep->fallback = reason;
    rep->diag = d;
    for (int k = 0; k < 3; ++k) rep->guess_err[k] = NAN;
    if (conv) {
        CHK(save_fields(n, g, n->fin));
        HIPCHK(nn::diff_norms3(n->guess, n->fin, (int64_t)hw, (int64_t)hw, n->npart, n->nout, s));
        double o[6];
        HIPCHK(hipMemcpyAsync(o, n->nout, sizeof(o), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        for (int k = 0; k < 3; ++k)
            rep->guess_err[k] = o[2 * k + 1] > 0 ? std::sqrt(o[2 * k] / o[2 * k + 1]) : std::sqrt(o[2 * k]);
    }
    rep->wall_s = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    return result;
}

}  // extern "C"
