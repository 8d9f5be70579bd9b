// Host side of the eLABSWE baseline (include/mlb.h, mlb_elab_*): nine
// distribution planes per buffer on the geometry, forcing and tiles of an
// existing grid.
#include <cmath>
#include <new>
#include <string>
#include <vector>

#include "mlb_runtime.h"

using namespace mlb;

struct mlb_elab {
    mlb_grid* g = nullptr;
    ElabDev D{};
    float* buf = nullptr;       // 2 x 9 planes, then 3 planes for macroscopic output
    TileDev* dtiles = nullptr;
    int ntiles = 0;
    int rd = 0;                 // buffer holding the current distributions
    int64_t step = 0;
};

extern "C" {

mlb_status mlb_elab_create(mlb_grid* g, double tau, mlb_elab** out)
{
    if (!g || !out) return fail(MLB_E_INVAL, "grid or out is NULL");
    *out = nullptr;
    if (!(tau > 0.5) || !std::isfinite(tau)) return fail(MLB_E_INVAL, "tau must be > 1/2");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    for (int k = 0; k < 4; ++k)
        if (g->p.edge[k] == MLB_EDGE_DEPTH || g->p.edge[k] == MLB_EDGE_DISCHARGE)
            return fail(MLB_E_INVAL, "the eLABSWE baseline supports wall and periodic edges only");
    if (g->hbar != MLB_HBAR_SEMI_IMPLICIT) return fail(MLB_E_INVAL, "the eLABSWE baseline uses Eq. h-bar");
    HIPCHK(hipSetDevice(g->ctx->device));
    mlb_elab* s = new (std::nothrow) mlb_elab();
    if (!s) return fail(MLB_E_NOMEM, "elab");
    s->g = g;
    const size_t plane = g->plane, stride = plane;
    hipError_t e = hipMalloc((void**)&s->buf, (2 * 9 * stride + 3 * plane) * sizeof(float));
    if (e != hipSuccess) { delete s; return fail(MLB_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); }
    std::vector<TileDev> t;
    grid_tiles(g, g->opts.tile_rows, t);
    s->ntiles = (int)t.size();
    e = hipMalloc((void**)&s->dtiles, t.size() * sizeof(TileDev));
    if (e == hipSuccess)
        e = hipMemcpyAsync(s->dtiles, t.data(), t.size() * sizeof(TileDev), hipMemcpyHostToDevice, g->ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(s->buf); (void)hipFree(s->dtiles); delete s;
        return fail(MLB_E_DEVICE, std::string("tiles: ") + hipGetErrorString(e));
    }
    ElabDev& D = s->D;
    D.f[0] = s->buf;
    D.f[1] = s->buf + 9 * stride;
    D.H = g->H;
    D.mask = g->dmask;
    D.plane = (int64_t)stride;
    D.nx = g->p.nx; D.ny = g->p.ny; D.ld = g->ld;
    D.per_x = g->p.edge[MLB_W] == MLB_EDGE_PERIODIC;
    D.per_y = g->p.edge[MLB_S] == MLB_EDGE_PERIODIC;
    const double ev = g->e, e2 = ev * ev, gr = g->p.g;
    D.e = (float)ev;
    D.tx = (float)g->tx; D.ty = (float)g->ty; D.cb = (float)g->cb; D.om = (float)g->p.omega;
    D.cfp = (float)(g->dt / (2.0 * ev));
    D.g6 = (float)(gr / (6.0 * e2));
    D.c6 = (float)(1.0 / (6.0 * e2));
    D.c3 = (float)(1.0 / (3.0 * ev));
    D.c2 = (float)(1.0 / (2.0 * e2));
    D.gb = (float)(gr / (2.0 * e2));
    D.rtau = (float)(1.0 / tau);
    e = launch_elab_init(D, g->eta[g->cur], g->qx[g->cur], g->qy[g->cur], g->ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(g->ctx->stream);
    if (e != hipSuccess) {
        (void)hipFree(s->buf); (void)hipFree(s->dtiles); delete s;
        return fail(MLB_E_DEVICE, std::string("init: ") + hipGetErrorString(e));
    }
    s->step = g->step;
    g->elab_refs++;
    *out = s;
    return MLB_OK;
}

mlb_status mlb_elab_step(mlb_elab* s, int64_t nsteps)
{
    if (!s) return fail(MLB_E_INVAL, "elab is NULL");
    if (nsteps < 0) return fail(MLB_E_INVAL, "nsteps < 0");
    mlb_ctx* c = s->g->ctx;
    HIPCHK(hipSetDevice(c->device));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    for (int64_t i = 0; i < nsteps; ++i) {
        HIPCHK(launch_elab_step(s->D, s->dtiles, s->ntiles, s->rd, c->stream));
        s->rd ^= 1;
    }
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    c->timed = true;
    s->step += nsteps;
    return MLB_OK;
}

mlb_status mlb_elab_get_state(mlb_elab* s, double* h, double* hu, double* hv, int64_t ld)
{
    if (!s) return fail(MLB_E_INVAL, "elab is NULL");
    mlb_grid* g = s->g;
    if (ld < g->p.nx) return fail(MLB_E_INVAL, "ld < nx");
    mlb_ctx* c = g->ctx;
    HIPCHK(hipSetDevice(c->device));
    const size_t plane = g->plane;
    float* m = s->buf + 18 * (size_t)s->D.plane;
    HIPCHK(launch_elab_macro(s->D, s->rd, m, m + plane, m + 2 * plane, c->stream));
    std::vector<float> v(3 * plane);
    HIPCHK(hipMemcpyAsync(v.data(), m, v.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    for (int j = 0; j < g->p.ny; ++j)
        for (int i = 0; i < g->p.nx; ++i) {
            const size_t o = (size_t)j * g->ld + i, d = (size_t)j * ld + i;
            if (h) h[d] = g->Hd[o] + (double)v[o];
            if (hu) hu[d] = v[plane + o];
            if (hv) hv[d] = v[2 * plane + o];
        }
    return MLB_OK;
}

mlb_status mlb_elab_get_dist_device(mlb_elab* s, float* f)
{
    if (!s || !f) return fail(MLB_E_INVAL, "NULL argument");
    mlb_grid* g = s->g;
    HIPCHK(hipSetDevice(g->ctx->device));
    HIPCHK(launch_elab_dist(s->D, s->rd, f, g->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_elab_destroy(mlb_elab* s)
{
    if (!s) return fail(MLB_E_INVAL, "elab is NULL");
    (void)hipSetDevice(s->g->ctx->device);
    (void)hipStreamSynchronize(s->g->ctx->stream);
    (void)hipFree(s->buf);
    (void)hipFree(s->dtiles);
    s->g->elab_refs--;
    delete s;
    return MLB_OK;
}

}  // extern "C"
