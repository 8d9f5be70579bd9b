// Host runtime behind the C ABI of include/mlb.h: contexts, grids, batches,
// parameter derivation and validation, tile plans, hipGraph step chunks,
// FP64 diagnostics.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <memory>
#include <string>
#include <thread>
#include <vector>

#include "mlb_runtime.h"

using namespace mlb;

namespace mlb {

namespace {
thread_local std::string g_err;
}

mlb_status fail(mlb_status s, const std::string& msg)
{
    g_err = msg;
    return s;
}

}  // namespace mlb

namespace {

inline bool is_open(int k) { return k == MLB_EDGE_DEPTH || k == MLB_EDGE_DISCHARGE; }
inline size_t align_up(size_t v, size_t a) { return (v + a - 1) / a * a; }
inline bool has_open_edge(const mlb_grid* g)
{
    for (int k = 0; k < 4; ++k)
        if (is_open(g->p.edge[k])) return true;
    return false;
}

}  // namespace

namespace {

// ------------------------------------------------------------------ helpers
BasinDev make_basin(const mlb_grid* g, int swap)
{
    BasinDev b{};
    for (int k = 0; k < 2; ++k) { b.eta[k] = g->eta[k]; b.qx[k] = g->qx[k]; b.qy[k] = g->qy[k]; }
    b.H = g->H;
    b.mask = g->dmask;
    const bool imp = g->hbar == MLB_HBAR_IMPLICIT && g->dcoef;
    b.cw = imp ? g->dcoef : nullptr;
    b.ckx = imp ? g->dcoef + g->plane : nullptr;
    b.cky = imp ? g->dcoef + 2 * g->plane : nullptr;
    for (int k = 0; k < 2; ++k) b.etal[k] = g->etal ? g->etal + k * g->plane : nullptr;
    b.stepc = g->stepc;
    b.dres = g->dres;
    b.nx = g->p.nx; b.ny = g->p.ny; b.ld = g->ld;
    b.swap = swap;
    b.per_x = g->p.edge[MLB_W] == MLB_EDGE_PERIODIC;
    b.per_y = g->p.edge[MLB_S] == MLB_EDGE_PERIODIC;
    for (int k = 0; k < 4; ++k) b.kind[k] = g->p.edge[k];
    b.extrap = g->p.extrap_order;
    const double e = g->e, dt = g->dt, gr = g->p.g, e2 = e * e;
    b.e = (float)e;
    // (+ 0.0f: a negative zero becomes +0, so that adding the zero Coriolis
    // term of Omega = 0 never changes a bit and the kernels may omit it)
    b.tpx = (float)(0.5 * dt * g->tx) + 0.0f;
    b.tpy = (float)(0.5 * dt * g->ty) + 0.0f;
    b.cfr = (float)(0.5 * dt * g->cb);
    b.omh = (float)(0.5 * dt * g->p.omega);
    b.c3e = (float)(1.0 / (3.0 * e));
    b.ckk = (float)(2.0 / (3.0 * e2));
    b.c6 = (float)(1.0 / (6.0 * e2));
    b.c12 = (float)(1.0 / (12.0 * e2));
    b.c4 = (float)(1.0 / (4.0 * e2));
    b.cma = (float)(gr / (6.0 * e2));
    b.cmd = (float)(gr / (24.0 * e2));
    b.cqa = (float)(gr / (6.0 * e));
    b.cqd = (float)(gr / (24.0 * e));
    b.dt = dt;
    for (int k = 0; k < 4; ++k) {
        b.bc_qx[k] = (float)g->bc_qx[k];
        b.bc_qy[k] = (float)g->bc_qy[k];
        b.bc_hmean[k] = g->bc_hmean[k];
        b.bc_amp[k] = g->bc_amp[k];
        b.bc_om[k] = g->bc_om[k];
        b.bc_phase[k] = g->bc_phase[k];
    }
    return b;
}

// Mask classification of a tile: TILE_MASKED when its window holds a WALL or
// SOLID node; false when every node it owns is SOLID (the tile has nothing
// to write and is left out).  The window is what the kernel loads, wrapped or
// clamped: one-step tiles columns x0-1 .. x0+62 and rows y0-1 .. y0+rows,
// two-step tiles columns x0-2 .. x0+61 and rows y0-2 .. y0+rows+1.
bool classify_tile(const mlb_grid* g, TileDev& t, int strip)
{
    const int halo = strip == kStripOut2 ? 2 : 1;
    const int nx = g->p.nx, ny = g->p.ny, ld = g->ld;
    const bool px = g->p.edge[MLB_W] == MLB_EDGE_PERIODIC, py = g->p.edge[MLB_S] == MLB_EDGE_PERIODIC;
    auto wrap = [](int v, int n, bool per) { return per ? ((v % n) + n) % n : std::min(std::max(v, 0), n - 1); };
    const uint8_t* m = g->hmask.data();
    bool any = false, owned_water = false;
    for (int r = t.y0 - halo; r <= t.y0 + t.rows + halo - 1; ++r) {
        const int rr = wrap(r, ny, py);
        for (int x = t.x0 - halo; x < t.x0 - halo + kWave; ++x) {
            const uint8_t k = m[(size_t)rr * ld + wrap(x, nx, px)];
            any |= k != NODE_FLUID;
            const bool own = x >= t.x0 && x < t.x0 + strip && x >= t.xo && x < nx && r >= t.yo &&
                             r < t.y0 + t.rows;
            owned_water |= own && k != NODE_SOLID;
        }
    }
    if (any) t.flags |= TILE_MASKED;
    return owned_water;
}

#ifndef MLB_COSTLY_FIRST
#define MLB_COSTLY_FIRST 1
#endif

// A tile whose window reaches a non-periodic edge, or holds a WALL or SOLID
// node: it takes the kernels' boundary path.
bool tile_costly(const mlb_grid* g, const TileDev& t, int strip)
{
    const int k = strip == kStripOut2 ? 2 : 1, nx = g->p.nx, ny = g->p.ny;
    const bool px = g->p.edge[MLB_W] == MLB_EDGE_PERIODIC, py = g->p.edge[MLB_S] == MLB_EDGE_PERIODIC;
    return (t.flags & TILE_MASKED) || (!px && (t.x0 < k || t.x0 + strip + k > nx)) ||
           (!py && (t.y0 < k || t.y0 + t.rows + k > ny));
}

// Wave tiles of one basin: strips of `strip` output columns (62 for one step
// per pass, 60 for two), tiles of `rows` rows.  The last strip / tile is
// shifted inward so that edge extrapolation always finds its inner nodes in
// the same tile; it then stores only what it owns.  Two-step tiles never
// start at row 1: their first stage would then compute row 0 of an open S
// edge, which waits for rows 1 and 2 (such a tile starts at row 0 instead).
// With a mask, tiles are classified by classify_tile.
void make_tiles(const mlb_grid* g, int basin, int rows, std::vector<TileDev>& out, int strip,
                bool costly_first = true)
{
    // List order = dispatch order: row band by row band, so one workgroup's
    // waves take neighbouring strips of one band (contiguous row segments).
    // Grouping vertically adjacent tiles per workgroup instead was measured
    // 5 % slower on the 4096^2 channel, and giving each XCD (the dispatcher
    // deals workgroups to the eight XCDs in turn) one contiguous run of the
    // list, so that neighbouring tiles share an L2, 8 % slower (two steps per
    // pass) and 9 % slower (one step); also with the costly tiles split
    // evenly over the XCDs ahead of each XCD's slab of bands: 288 against
    // 312-318 GLUPS at 26-row tiles.
    const int nx = g->p.nx, ny = g->p.ny;
    const int ty = std::max(4, rows);
    const size_t first = out.size();
    for (int yo = 0; yo < ny; yo += ty) {
        int y0 = std::min(yo, std::max(0, ny - ty));
        if (strip == kStripOut2 && y0 == 1) y0 = 0;
        const int yend = std::min(yo + ty, ny);
        for (int xo = 0; xo < nx; xo += strip) {
            TileDev t{};
            t.basin = basin;
            t.xo = xo;
            t.x0 = std::min(xo, std::max(0, nx - strip));
            t.yo = yo;
            t.y0 = y0;
            t.rows = yend - y0;
            if (!g->hmask.empty() && !classify_tile(g, t, strip)) continue;
            out.push_back(t);
        }
    }
#if MLB_COSTLY_FIRST
    // Tiles on an edge or with a mask cost up to a few interior tiles each:
    // dispatched first, they overlap the bulk of the pass instead of running
    // alone at its end (tiles are independent within a pass).  Measured on the
    // 4096^2 channel: 287 -> 310 GLUPS with two steps per pass.
    if (costly_first)
        std::stable_partition(out.begin() + first, out.end(),
                              [&](const TileDev& t) { return tile_costly(g, t, strip); });
#else
    (void)first; (void)costly_first;
#endif
}

mlb_status check_stream(mlb_ctx* c)
{
    HIPCHK(hipSetDevice(c->device));
    return MLB_OK;
}

mlb_status plan_alloc(mlb_ctx* c, Plan& P)
{
    const size_t nb = P.hb.size(), nt = P.ht.size();
    // partials of a checked pass: one set per tile of either list
    const size_t np = std::max<size_t>(1, std::max(nt, P.ht2.size()));
    HIPCHK(hipMalloc(&P.db, nb * sizeof(BasinDev)));
    HIPCHK(hipMalloc(&P.dt, nt * sizeof(TileDev)));
    HIPCHK(hipMalloc(&P.dpart, np * kPartials * sizeof(double)));
    HIPCHK(hipMalloc(&P.dout, nb * 8 * sizeof(double)));
    HIPCHK(hipHostMalloc(&P.hout, nb * 8 * sizeof(double), hipHostMallocDefault));
    HIPCHK(hipMalloc(&P.dsync, sizeof(SyncState)));
    HIPCHK(hipHostMalloc(&P.herr, sizeof(int32_t), hipHostMallocDefault));
    HIPCHK(hipMemsetAsync(P.dsync, 0, sizeof(SyncState), c->stream));
    P.sync_base = 0;
    P.coop_failed = false;
    HIPCHK(hipMemcpyAsync(P.dt, P.ht.data(), nt * sizeof(TileDev), hipMemcpyHostToDevice, c->stream));
    if (!P.ht2.empty()) {
        HIPCHK(hipMalloc(&P.dt2, P.ht2.size() * sizeof(TileDev)));
        HIPCHK(hipMemcpyAsync(P.dt2, P.ht2.data(), P.ht2.size() * sizeof(TileDev), hipMemcpyHostToDevice,
                              c->stream));
    }
    HIPCHK(hipMemcpyAsync(P.db, P.hb.data(), nb * sizeof(BasinDev), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    P.built = true;
    return MLB_OK;
}

mlb_status upload_basins(mlb_ctx* c, Plan& P)
{
    HIPCHK(hipMemcpyAsync(P.db, P.hb.data(), P.hb.size() * sizeof(BasinDev), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return MLB_OK;
}

// Single-grid plan.
mlb_status grid_plan(mlb_grid* g)
{
    mlb_ctx* c = g->ctx;
    if (g->stale_plan || !g->plan.built) {
        g->plan.release();
        g->plan.hb.assign(1, make_basin(g, g->cur));
        g->plan.parity = 0;
        g->plan.ht.clear();
        g->plan.ht2.clear();
        make_tiles(g, 0, g->opts.tile_rows, g->plan.ht, kStripOut);
        // the compensated surface runs one step per pass
        const bool one = g->etal != nullptr;
        if (g->opts.tblock == 2 && !one) make_tiles(g, 0, g->opts.tile_rows, g->plan.ht2, kStripOut2);
        g->plan.hb[0].first_tile = 0;
        g->plan.hb[0].ntiles = (int)g->plan.ht.size();
        g->plan.hb[0].first_tile2 = 0;
        g->plan.hb[0].ntiles2 = (int)g->plan.ht2.size();
        g->plan.masked = g->dmask != nullptr;
        g->plan.implicit = g->hbar == MLB_HBAR_IMPLICIT;
        g->plan.comp = g->etal != nullptr;
        g->plan.closed = !has_open_edge(g);
        CHK(plan_alloc(c, g->plan));
        g->stale_plan = false;
        g->dirty = false;
    } else if (g->dirty) {
        BasinDev b = make_basin(g, g->plan.parity ^ g->cur);
        b.first_tile = 0;
        b.ntiles = (int)g->plan.ht.size();
        b.first_tile2 = 0;
        b.ntiles2 = (int)g->plan.ht2.size();
        g->plan.hb[0] = b;
        CHK(upload_basins(c, g->plan));
        g->dirty = false;
    }
    return MLB_OK;
}

// A persistent launch gives up at a pass barrier when a bounded wait runs
// out; its passes are then incomplete and later persistent launches of the
// plan do nothing.  After each persistent launch the flag is copied to the
// host in stream order (watch_abort); the calls that hand out state or
// diagnostics check it (check_abort, after the stream has drained), report
// MLB_E_DEVICE and clear the flag, so that the state can be set again.
mlb_status watch_abort(mlb_ctx* c, Plan& P)
{
    HIPCHK(hipMemcpyAsync(P.herr, &P.dsync->err, sizeof(int32_t), hipMemcpyDeviceToHost, c->stream));
    if (!P.err_pending) {
        P.err_pending = true;
        P.watch = c;
        c->watch.push_back(&P);
    }
    return MLB_OK;
}

mlb_status check_abort(mlb_ctx* c, Plan& P)
{
    if (!P.err_pending) return MLB_OK;
    HIPCHK(hipStreamSynchronize(c->stream));
    plan_unwatch(P);
    if (*(volatile int32_t*)P.herr) {
        *P.herr = 0;
        HIPCHK(hipMemsetAsync(P.dsync, 0, sizeof(SyncState), c->stream));
        HIPCHK(hipStreamSynchronize(c->stream));
        P.sync_base = 0;
        P.wq[0].release();   // epochs of an abandoned launch: rebuilt on next use
        P.wq[1].release();
        return fail(MLB_E_DEVICE, "a persistent launch timed out at a pass barrier; the state is incomplete");
    }
    return MLB_OK;
}

// The same without waiting: reports a give-up whose flag copy has already
// landed (calls that only enqueue work check this way).
mlb_status peek_abort(mlb_ctx* c, Plan& P)
{
    if (P.err_pending && *(volatile int32_t*)P.herr) return check_abort(c, P);
    return MLB_OK;
}

// Dependency lists of a plan's tile list for work-queue launches.  A tile's
// owned nodes form a (strip, band) cell of its basin; its window is what its
// wave loads (one-step tiles columns x0-1 .. x0+62 and rows y0-1 .. y0+rows,
// two-step tiles columns x0-2 .. x0+61 and rows y0-2 .. y0+rows+1, wrapped on
// periodic axes, clamped otherwise).  W(t) = the tiles owning a node of t's
// window; D(t) = W(t) plus every u with t in W(u) (u reads what t writes).
// An item (p, t) waits until every tile of D(t) has completed pass p - 1:
// its reads then see pass p - 1's values, and no tile still reads the
// buffer it overwrites.
// false when some tile has more than kWave dependencies.
bool wq_dependencies(const std::vector<BasinDev>& hb, const std::vector<TileDev>& tl, int kind,
                     std::vector<int32_t>& off, std::vector<int32_t>& nbr)
{
    const int nt = (int)tl.size(), strip = kind == 2 ? kStripOut2 : kStripOut, halo = kind == 2 ? 2 : 1;
    std::vector<std::vector<int32_t>> dep(nt);
    int i0 = 0;
    while (i0 < nt) {   // the tiles of one basin are contiguous in the list
        const int b = tl[i0].basin;
        int i1 = i0;
        while (i1 < nt && tl[i1].basin == b) ++i1;
        const BasinDev& B = hb[b];
        const int nx = B.nx, ny = B.ny;
        int ty = ny;   // band height: the smallest positive first owned row
        for (int i = i0; i < i1; ++i)
            if (tl[i].yo > 0) ty = std::min(ty, tl[i].yo);
        const int ns = (nx + strip - 1) / strip, nb = (ny + ty - 1) / ty;
        std::vector<int32_t> cell((size_t)ns * nb, -1);
        for (int i = i0; i < i1; ++i) cell[(size_t)(tl[i].yo / ty) * ns + tl[i].xo / strip] = i;
        auto wrap = [](int v, int n, int per) { return per ? ((v % n) + n) % n : std::min(std::max(v, 0), n - 1); };
        std::vector<int> sx, sy;
        for (int i = i0; i < i1; ++i) {
            const TileDev& T = tl[i];
            sx.clear(); sy.clear();
            for (int x = T.x0 - halo; x < T.x0 - halo + kWave; ++x) sx.push_back(wrap(x, nx, B.per_x) / strip);
            for (int y = T.y0 - halo; y <= T.y0 + T.rows + halo - 1; ++y) sy.push_back(wrap(y, ny, B.per_y) / ty);
            std::sort(sx.begin(), sx.end()); sx.erase(std::unique(sx.begin(), sx.end()), sx.end());
            std::sort(sy.begin(), sy.end()); sy.erase(std::unique(sy.begin(), sy.end()), sy.end());
            for (int yb : sy)
                for (int xs : sx) {
                    const int u = cell[(size_t)yb * ns + xs];
                    if (u < 0) continue;   // a tile left out (every node it would own is SOLID)
                    dep[i].push_back(u);
                    dep[u].push_back(i);
                }
        }
        i0 = i1;
    }
    off.assign(nt + 1, 0);
    nbr.clear();
    for (int i = 0; i < nt; ++i) {
        auto& d = dep[i];
        d.push_back(i);
        std::sort(d.begin(), d.end());
        d.erase(std::unique(d.begin(), d.end()), d.end());
        if (d.size() > (size_t)kWave) return false;
        off[i + 1] = off[i] + (int32_t)d.size();
        nbr.insert(nbr.end(), d.begin(), d.end());
    }
    return true;
}

mlb_status build_workqueue(mlb_ctx* c, Plan& P, int kind)
{
    WqBuf& W = P.wq[kind - 1];
    const int nt = (int)(kind == 2 ? P.ht2 : P.ht).size();
    std::vector<int32_t> off, nbr;
    if (!wq_dependencies(P.hb, kind == 2 ? P.ht2 : P.ht, kind, off, nbr)) { W.failed = true; return MLB_OK; }
    W.release();
    HIPCHK(hipMalloc((void**)&W.q.cursor, sizeof(uint32_t)));
    HIPCHK(hipMalloc((void**)&W.q.epoch, std::max(1, nt) * sizeof(uint32_t)));
    HIPCHK(hipMalloc((void**)&W.q.nbr_off, off.size() * sizeof(int32_t)));
    HIPCHK(hipMalloc((void**)&W.q.nbr, std::max<size_t>(1, nbr.size()) * sizeof(int32_t)));
    HIPCHK(hipMalloc((void**)&W.q.base, P.hb.size() * sizeof(int64_t)));
    HIPCHK(hipMemsetAsync(W.q.epoch, 0, std::max(1, nt) * sizeof(uint32_t), c->stream));
    HIPCHK(hipMemcpyAsync((void*)W.q.nbr_off, off.data(), off.size() * sizeof(int32_t), hipMemcpyHostToDevice,
                          c->stream));
    HIPCHK(hipMemcpyAsync((void*)W.q.nbr, nbr.data(), nbr.size() * sizeof(int32_t), hipMemcpyHostToDevice, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    W.q.err = &P.dsync->err;
    W.passes = 0;
    W.ok = true;
    return MLB_OK;
}

// Launch n steps of a plan; the last one reduces into partials when diag.
// Advances the plan parity per launch; graph chunks replay when aligned.
// Dynamic LDS per step workgroup that leaves room for at most
// o.blocks_per_cu resident workgroups on a CU (0: no cap).
unsigned dyn_lds_for(const mlb_ctx* c, const mlb_exec_opts& o)
{
    if (o.blocks_per_cu <= 0 || c->lds_per_cu <= 0) return 0;
    // rounded down to 2 KiB so that allocation granularity never lets fewer fit
    const unsigned per = (unsigned)(c->lds_per_cu / o.blocks_per_cu) / 2048u * 2048u;
    return (unsigned)(o.blocks_per_cu + 1) * per > (unsigned)c->lds_per_cu ? per : 0u;
}

mlb_status enqueue_steps(mlb_ctx* c, Plan& P, const mlb_exec_opts& o, int64_t n, bool diag_last,
                         int64_t* launches)
{
    const int nt1 = (int)P.ht.size(), nt2 = (int)P.ht2.size();
    const unsigned dyn = dyn_lds_for(c, o);
    // Two steps per launch when the plan has the two-step tiles; an odd count
    // takes one single step first.  A checked call (diag_last) ends with a
    // checked pass of the same kind: its last step is reduced into the tile
    // partials (residual against the level before it, which a two-step pass
    // holds in registers) and finalised into every basin's result slot.
    const int kind = (o.tblock == 2 && P.dt2) ? 2 : 1;
    int64_t nl = 0;
    auto eager = [&](int k, bool diag) -> mlb_status {
        HIPCHK(launch_step(P.db, k == 2 ? P.dt2 : P.dt, k == 2 ? nt2 : nt1, P.parity, P.dpart, diag ? 1 : 0, k,
                           P.masked ? 1 : 0, P.implicit ? 1 : 0, P.comp ? 1 : 0, P.closed ? 1 : 0, dyn,
                           c->stream));
        P.parity ^= 1;
        ++nl;
        return MLB_OK;
    };
    int64_t lead = kind == 2 ? (n & 1) : 0;   // single steps before the passes of `kind`
    int64_t multi = kind == 2 ? n / 2 : n;     // passes of `kind`
    int closing = 0;                           // steps of the closing checked pass
    if (diag_last && n > 0) {
        if (multi > 0) { closing = kind; --multi; }
        else { closing = 1; --lead; }
    }
    for (int64_t i = 0; i < lead; ++i) CHK(eager(1, false));
    HIPCHK(hipEventRecord(c->ev2, c->stream));
    c->bulk_passes = multi;
    c->bulk_kind = kind;
    // work queue: all `multi` passes in persistent launches ordered per tile
    // by epoch flags (not for the implicit link depth or the compensated
    // surface: those basins use ordinary launches)
    if (o.persistent == 2 && multi > 0 && !P.implicit && !P.comp) {
        WqBuf& W = P.wq[kind - 1];
        if (!W.ok && !W.failed) CHK(build_workqueue(c, P, kind));
        if (W.ok) {
            const int nt = kind == 2 ? nt2 : nt1;
            int64_t nblk = (int64_t)workqueue_occupancy(kind, P.masked ? 1 : 0, P.closed ? 1 : 0) * c->ncu;
            if (o.blocks_per_cu > 0) nblk = std::min<int64_t>(nblk, (int64_t)o.blocks_per_cu * c->ncu);
            // items are 32-bit: at most 2^31 per launch
            const int64_t maxp = std::max<int64_t>(1, ((int64_t)1 << 31) / std::max(1, nt));
            while (multi > 0) {
                const int np = (int)std::min<int64_t>(multi, std::min<int64_t>(maxp, 1 << 16));
                // about one wave per tile of a pass: every wave then works or
                // waits for the pass before, and few waves poll at once
                const int nb = (int)std::max<int64_t>(
                    1, std::min<int64_t>(nblk, ((int64_t)nt + kBlock / kWave - 1) / (kBlock / kWave)));
                HIPCHK(launch_workqueue(P.db, (int)P.hb.size(), kind == 2 ? P.dt2 : P.dt, nt, P.parity, np, kind,
                                        P.masked ? 1 : 0, P.closed ? 1 : 0, W.q, W.passes, c->spin_limit, nb, dyn,
                                        c->stream));
                W.passes += (uint32_t)np;
                P.parity ^= np & 1;
                nl += np;
                multi -= np;
                CHK(watch_abort(c, P));
            }
        }
    }
    // persistent: all `multi` passes in cooperative launches with grid barriers
    // (not for the implicit link depth: those basins use ordinary launches)
    if (o.persistent == 1 && multi > 0 && !P.coop_failed && !P.implicit && !P.comp) {
        const int nt = kind == 2 ? nt2 : nt1;
        const int nblk = (nt + kBlock / kWave - 1) / (kBlock / kWave);
        if (persistent_capacity(kind, P.masked ? 1 : 0, c->ncu) < nblk) {
            P.coop_failed = true;
        } else {
            while (multi > 0) {
                const int np = (int)std::min<int64_t>(multi, 1 << 12);
                const hipError_t e = launch_persistent(P.db, kind == 2 ? P.dt2 : P.dt, nt, P.parity, np, kind,
                                                       P.masked ? 1 : 0, P.dsync, P.sync_base, c->spin_limit, c->stream);
                if (e != hipSuccess) {
                    (void)hipGetLastError();
                    P.coop_failed = true;   // ordinary launches for the rest
                    break;
                }
                P.sync_base += (uint64_t)np * (uint64_t)nblk;
                P.parity ^= np & 1;
                nl += np;
                multi -= np;
                CHK(watch_abort(c, P));
            }
        }
    }
    // graphs hold an even number of launches, so the parity they start from
    // recurs; a call shorter than one chunk captures a graph of its own length
    int glaunch = kind == 2 ? std::max(2, (o.graph_chunk / 2) & ~1) : std::max(2, o.graph_chunk & ~1);
    if (multi < glaunch && multi >= 4) glaunch = (int)(multi & ~(int64_t)1);
    if (o.use_graph && multi >= glaunch) {
        if (!P.gexec || P.gsteps != glaunch || P.gkind != kind || P.gdyn != dyn) {
            if (P.gexec) { (void)hipGraphExecDestroy(P.gexec); P.gexec = nullptr; }
            if (P.graph) { (void)hipGraphDestroy(P.graph); P.graph = nullptr; }
            HIPCHK(hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
            int par = P.parity;
            hipError_t le = hipSuccess;
            for (int i = 0; i < glaunch && le == hipSuccess; ++i) {
                le = launch_step(P.db, kind == 2 ? P.dt2 : P.dt, kind == 2 ? nt2 : nt1, par, P.dpart, 0, kind,
                                 P.masked ? 1 : 0, P.implicit ? 1 : 0, P.comp ? 1 : 0, P.closed ? 1 : 0, dyn,
                                 c->stream);
                par ^= 1;
            }
            hipGraph_t gr = nullptr;
            hipError_t ee = hipStreamEndCapture(c->stream, &gr);
            if (le != hipSuccess) return fail(MLB_E_DEVICE, std::string("capture: ") + hipGetErrorString(le));
            if (ee != hipSuccess) return fail(MLB_E_DEVICE, std::string("end capture: ") + hipGetErrorString(ee));
            P.graph = gr;
            HIPCHK(hipGraphInstantiate(&P.gexec, P.graph, nullptr, nullptr, 0));
            P.gsteps = glaunch;
            P.gkind = kind;
            P.gparity = P.parity;
            P.gdyn = dyn;
        }
        if (P.parity != P.gparity) {
            CHK(eager(kind, false));
            --multi;
        }
        while (multi >= glaunch) {
            HIPCHK(hipGraphLaunch(P.gexec, c->stream));
            multi -= glaunch;
            nl += glaunch;
        }
    }
    for (int64_t i = 0; i < multi; ++i) CHK(eager(kind, false));
    HIPCHK(hipEventRecord(c->ev3, c->stream));
    if (closing) {
        CHK(eager(closing, true));
        HIPCHK(launch_finalize(P.db, (int)P.hb.size(), P.dpart, P.dout, closing, c->stream));
    }
    if (launches) *launches = nl;
    return MLB_OK;
}

// Row pitch: nx rounded up to 64 floats (256 B), plus MLB_LD_PAD floats
// (build-time knob; breaks power-of-two pitches).
#ifndef MLB_LD_PAD
#define MLB_LD_PAD 0
#endif
int64_t row_pitch(int nx) { return (int64_t)align_up((size_t)nx, 64) + MLB_LD_PAD; }

mlb_status validate_params(const mlb_params* p)
{
    if (!p) return fail(MLB_E_INVAL, "params is NULL");
    const bool px = p->edge[MLB_W] == MLB_EDGE_PERIODIC, ex = p->edge[MLB_E] == MLB_EDGE_PERIODIC;
    const bool py = p->edge[MLB_S] == MLB_EDGE_PERIODIC, ey = p->edge[MLB_N] == MLB_EDGE_PERIODIC;
    for (int k = 0; k < 4; ++k)
        if (p->edge[k] < MLB_EDGE_WALL || p->edge[k] > MLB_EDGE_DISCHARGE)
            return fail(MLB_E_INVAL, "unknown edge kind");
    if (px != ex || py != ey) return fail(MLB_E_INVAL, "periodic edges must be set in pairs");
    const bool ox = is_open(p->edge[MLB_W]) || is_open(p->edge[MLB_E]);
    const bool oy = is_open(p->edge[MLB_S]) || is_open(p->edge[MLB_N]);
    if (ox && oy) return fail(MLB_E_INVAL, "two adjacent edges may not both be open");
    const int minx = px ? 3 : (ox ? 5 : 4), miny = py ? 3 : (oy ? 5 : 4);
    if (p->nx < minx || p->ny < miny) return fail(MLB_E_INVAL, "grid too small for its edges");
    // the kernels address a field plane with 32-bit byte offsets: the padded
    // plane (row pitch x ny) must hold fewer than 2^30 floats
    if ((int64_t)row_pitch(p->nx) * p->ny >= ((int64_t)1 << 30))
        return fail(MLB_E_INVAL, "grid too large: row pitch x ny must stay below 2^30 nodes");
    if (!(p->dx > 0) || !(p->nu > 0) || !(p->g > 0) || !(p->rho_w > 0))
        return fail(MLB_E_INVAL, "dx, nu, g and rho_w must be positive");
    if (p->extrap_order != 1 && p->extrap_order != 2) return fail(MLB_E_INVAL, "extrap_order must be 1 or 2");
    return MLB_OK;
}

size_t field_bytes(const mlb_params* p, int* ld_out)
{
    const int ld = (int)row_pitch(p->nx);
    if (ld_out) *ld_out = ld;
    return 256 + 7 * align_up((size_t)ld * p->ny * sizeof(float), 256);
}

// fn(j0, j1) over row ranges covering 0 .. ny-1, on up to 16 host threads for
// large grids (each row is converted independently, so the split does not
// change any value).
template <class F>
void for_rows(int ny, size_t nodes, F fn)
{
    const unsigned hw = std::thread::hardware_concurrency();
    const int nt = nodes < ((size_t)1 << 18) ? 1 : (int)std::min<unsigned>(16u, std::max(1u, hw));
    if (nt <= 1 || ny < 2 * nt) { fn(0, ny); return; }
    std::vector<std::thread> pool;
    const int per = (ny + nt - 1) / nt;
    for (int t = 1; t < nt; ++t) {
        const int j0 = t * per, j1 = std::min(ny, j0 + per);
        if (j0 < j1) pool.emplace_back(fn, j0, j1);
    }
    fn(0, std::min(ny, per));
    for (auto& th : pool) th.join();
}

mlb_status upload_host_state(mlb_grid* g, const double* h, const double* hu, const double* hv,
                             int64_t ld)
{
    const int nx = g->p.nx, ny = g->p.ny;
    const size_t n = (size_t)g->ld * ny;
    std::unique_ptr<float[]> e(new (std::nothrow) float[n]), a(new (std::nothrow) float[n]),
        b(new (std::nothrow) float[n]);
    std::unique_ptr<float[]> el(g->etal ? new (std::nothrow) float[n] : nullptr);
    if (!e || !a || !b || (g->etal && !el)) return fail(MLB_E_NOMEM, "host staging of the state");
    for_rows(ny, (size_t)nx * ny, [&](int j0, int j1) {
        for (int j = j0; j < j1; ++j) {
            for (int i = 0; i < nx; ++i) {
                const size_t s = (size_t)j * ld + i, d = (size_t)j * g->ld + i;
                const double ed = h ? h[s] - g->Hd[d] : 0.0;
                e[d] = (float)ed;
                if (g->etal) el[d] = (float)(ed - (double)e[d]);   // compensated surface: the remainder
                a[d] = hu ? (float)hu[s] : 0.f;
                b[d] = hv ? (float)hv[s] : 0.f;
            }
            for (int i = nx; i < g->ld; ++i) {   // row padding: zero
                const size_t d = (size_t)j * g->ld + i;
                e[d] = a[d] = b[d] = 0.f;
                if (g->etal) el[d] = 0.f;
            }
        }
    });
    const size_t bytes = n * sizeof(float);
    for (int k = 0; k < 2; ++k) {
        HIPCHK(hipMemcpyAsync(g->eta[k], e.get(), bytes, hipMemcpyHostToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qx[k], a.get(), bytes, hipMemcpyHostToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qy[k], b.get(), bytes, hipMemcpyHostToDevice, g->ctx->stream));
        if (g->etal)
            HIPCHK(hipMemcpyAsync(g->etal + k * g->plane, el.get(), bytes, hipMemcpyHostToDevice, g->ctx->stream));
    }
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    return MLB_OK;
}

// Sum of the still-water depth over the water (every node but SOLID ones):
// the mass diagnostic adds the reduced sum of eta to it.
double water_depth_sum(const mlb_grid* g)
{
    double sum = 0;
    for (int j = 0; j < g->p.ny; ++j)
        for (int i = 0; i < g->p.nx; ++i) {
            const size_t o = (size_t)j * g->ld + i;
            if (g->hmask.empty() || g->hmask[o] != NODE_SOLID) sum += g->Hd[o];
        }
    return sum;
}

// Static sums of the implicit link depth per node x, over its links a whose
// upstream node y = x - e_a is in the water (not past a non-periodic edge, not
// SOLID):  kappa = g/(2e^2) sum_a C_a (z_x - z_y),
//          kappa_v = g/(2e) sum_a C_a e^_a (z_x - z_y),  z_x - z_y = H_y - H_x,
// in FP64 from the depths as given; stored 1/(1+kappa), kappa_x, kappa_y (FP32).
mlb_status implicit_coeffs(mlb_grid* g)
{
    if (g->hbar != MLB_HBAR_IMPLICIT) return MLB_OK;
    // D2Q9 (Section 3): axis directions C = 1/3, diagonals C = 1/12, numbered
    // counter-clockwise from east
    static const int ex[9] = {0, 1, 1, 0, -1, -1, -1, 0, 1};
    static const int ey[9] = {0, 0, 1, 1, 1, 0, -1, -1, -1};
    static const double ca[9] = {0, 1.0 / 3, 1.0 / 12, 1.0 / 3, 1.0 / 12, 1.0 / 3, 1.0 / 12, 1.0 / 3, 1.0 / 12};
    const int nx = g->p.nx, ny = g->p.ny, ld = g->ld;
    const bool px = g->p.edge[MLB_W] == MLB_EDGE_PERIODIC, py = g->p.edge[MLB_S] == MLB_EDGE_PERIODIC;
    const double e = g->e, cm = g->p.g / (2.0 * e * e), cv = g->p.g / (2.0 * e);
    std::vector<float> w(3 * g->plane, 0.0f);
    float* kx = w.data() + g->plane;
    float* ky = w.data() + 2 * g->plane;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t o = (size_t)j * ld + i;
            double kap = 0, kvx = 0, kvy = 0;
            for (int a = 1; a <= 8; ++a) {
                int yi = i - ex[a], yj = j - ey[a];
                if (yi < 0 || yi >= nx) { if (!px) continue; yi = (yi + nx) % nx; }
                if (yj < 0 || yj >= ny) { if (!py) continue; yj = (yj + ny) % ny; }
                const size_t y = (size_t)yj * ld + yi;
                if (!g->hmask.empty() && g->hmask[y] == NODE_SOLID) continue;
                const double dz = g->Hd[y] - g->Hd[o];
                kap += cm * ca[a] * dz;
                kvx += cv * ca[a] * ex[a] * dz;
                kvy += cv * ca[a] * ey[a] * dz;
            }
            if (!(1.0 + kap > 0)) return fail(MLB_E_UNSTABLE, "implicit link depth: 1 + kappa <= 0 at a node");
            w[o] = (float)(1.0 / (1.0 + kap));
            kx[o] = (float)kvx;
            ky[o] = (float)kvy;
        }
    if (!g->dcoef) HIPCHK(hipMalloc((void**)&g->dcoef, w.size() * sizeof(float)));
    HIPCHK(hipMemcpyAsync(g->dcoef, w.data(), w.size() * sizeof(float), hipMemcpyHostToDevice, g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    g->dirty = true;
    return MLB_OK;
}

mlb_status set_step(mlb_grid* g, int64_t s)
{
    int64_t v[2] = {s, s};
    HIPCHK(hipMemcpyAsync(g->stepc, v, sizeof(v), hipMemcpyHostToDevice, g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    g->step = s;
    return MLB_OK;
}

void fill_diag(const mlb_grid* g, const double* o, mlb_diag_t* d)
{
    d->step = g->step;
    d->t = (double)g->step * g->dt;
    d->mass = (g->sumH + o[0]) * g->p.dx * g->p.dx;
    d->residual = o[1] > 0 ? std::sqrt(o[1]) / std::sqrt(o[2]) : 0.0;
    d->max_speed = o[4];
    d->nonfinite = (int64_t)o[3];
    d->e = g->e;
    d->dt = g->dt;
    d->gh_over_e2 = g->p.g * g->Hmax / (g->e * g->e);
    d->rle = o[4] * g->p.dx / g->p.nu;
}

// The finalised sums of a plan's last checked pass (P.dout) to the host.
mlb_status read_diag(mlb_ctx* c, Plan& P)
{
    HIPCHK(hipMemcpyAsync(P.hout, P.dout, P.hb.size() * 8 * sizeof(double), hipMemcpyDeviceToHost,
                          c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    return check_abort(c, P);
}

#define GRID_OK(g)                                                         \
    do {                                                                   \
        if (!(g)) return fail(MLB_E_INVAL, "grid is NULL");                \
        CHK(check_stream((g)->ctx));                                       \
    } while (0)

}  // namespace

namespace mlb {
void plan_unwatch(Plan& P)
{
    if (P.watch) {
        auto& w = P.watch->watch;
        w.erase(std::remove(w.begin(), w.end(), &P), w.end());
    }
    P.watch = nullptr;
    P.err_pending = false;
}
void grid_state_changed(mlb_grid* g) { g->diag_fresh = false; }
mlb_status grid_set_step(mlb_grid* g, int64_t s) { return set_step(g, s); }
// (band order: the eLABSWE kernel measured 2.5 % slower with its edge tiles first)
void grid_tiles(const mlb_grid* g, int rows, std::vector<TileDev>& out) { make_tiles(g, 0, rows, out, kStripOut, false); }
}  // namespace mlb

// ====================================================================== C ABI
extern "C" {

const char* mlb_status_str(mlb_status s)
{
    switch (s) {
    case MLB_OK: return "ok";
    case MLB_E_INVAL: return "invalid argument";
    case MLB_E_NOMEM: return "out of memory";
    case MLB_E_DEVICE: return "device error";
    case MLB_E_UNSTABLE: return "unstable parameters (g H > e^2)";
    case MLB_E_NONFINITE: return "non-finite value or dry node";
    case MLB_E_STATE: return "invalid state for this call";
    case MLB_E_NOTCONVERGED: return "not converged";
    case MLB_E_STALLED: return "residual stalled";
    }
    return "unknown status";
}

const char* mlb_last_error(void) { return mlb::g_err.c_str(); }

mlb_status mlb_ctx_create(int device, void* hip_stream, mlb_ctx** out)
{
    if (!out) return fail(MLB_E_INVAL, "out is NULL");
    *out = nullptr;
    int n = 0;
    HIPCHK(hipGetDeviceCount(&n));
    if (device < 0 || device >= n) return fail(MLB_E_INVAL, "no such device");
    HIPCHK(hipSetDevice(device));
    CHK(noalloc_setup(device));
    mlb_ctx* c = new (std::nothrow) mlb_ctx();
    if (!c) return fail(MLB_E_NOMEM, "ctx");
    c->device = device;
    if (hip_stream) {
        c->stream = (hipStream_t)hip_stream;
    } else {
        hipError_t e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (e != hipSuccess) { delete c; return fail(MLB_E_DEVICE, hipGetErrorString(e)); }
        c->own_stream = true;
    }
    (void)hipDeviceGetAttribute(&c->ncu, hipDeviceAttributeMultiprocessorCount, device);
    if (c->ncu <= 0) c->ncu = 256;
    (void)hipDeviceGetAttribute(&c->lds_per_cu, hipDeviceAttributeMaxSharedMemoryPerMultiprocessor, device);
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, device) == hipSuccess) c->arch = prop.gcnArchName;
    if (c->arch.empty()) c->arch = "gpu";
    for (auto& ch : c->arch) if (ch == ' ' || ch == ':') ch = '_';
    (void)hipEventCreate(&c->ev0);
    (void)hipEventCreate(&c->ev1);
    (void)hipEventCreate(&c->ev2);
    (void)hipEventCreate(&c->ev3);
    // bounded wait of persistent launches (polls); a small value forces the
    // timeout path from the host
    if (const char* sl = std::getenv("MLB_SPIN_LIMIT")) {
        const long v = std::strtol(sl, nullptr, 10);
        if (v >= 0 && v < (1L << 30)) c->spin_limit = (int)v;
    }
    *out = c;
    return MLB_OK;
}

mlb_status mlb_ctx_destroy(mlb_ctx* c)
{
    if (!c) return fail(MLB_E_INVAL, "ctx is NULL");
    if (c->live) return fail(MLB_E_STATE, "grids or batches still alive");
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    if (c->ev0) (void)hipEventDestroy(c->ev0);
    if (c->ev1) (void)hipEventDestroy(c->ev1);
    if (c->ev2) (void)hipEventDestroy(c->ev2);
    if (c->ev3) (void)hipEventDestroy(c->ev3);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
    return MLB_OK;
}

mlb_status mlb_set_stall_checks(mlb_ctx* c, int32_t checks)
{
    if (!c || checks < 0) return fail(MLB_E_INVAL, "bad stall setting");
    c->stall_checks = checks;
    return MLB_OK;
}

mlb_status mlb_ctx_sync(mlb_ctx* c)
{
    if (!c) return fail(MLB_E_INVAL, "ctx is NULL");
    CHK(check_stream(c));
    HIPCHK(hipStreamSynchronize(c->stream));
    mlb_status st = MLB_OK;
    while (!c->watch.empty()) {   // every watched plan is checked (and cleared)
        const mlb_status s1 = check_abort(c, *c->watch.back());
        if (st == MLB_OK) st = s1;
    }
    if (st != MLB_OK) return fail(st, "a persistent launch timed out at a pass barrier; the state is incomplete");
    return MLB_OK;
}

mlb_status mlb_grid_workspace_bytes(const mlb_params* p, size_t* bytes)
{
    CHK(validate_params(p));
    if (!bytes) return fail(MLB_E_INVAL, "bytes is NULL");
    *bytes = field_bytes(p, nullptr);
    return MLB_OK;
}

mlb_status mlb_grid_create(mlb_ctx* c, const mlb_params* p, void* ws, size_t ws_bytes, mlb_grid** out)
{
    if (!c || !out) return fail(MLB_E_INVAL, "ctx or out is NULL");
    *out = nullptr;
    CHK(validate_params(p));
    CHK(check_stream(c));
    int ld = 0;
    const size_t need = field_bytes(p, &ld);
    if (ws && (ws_bytes < need || ((uintptr_t)ws & 255)))
        return fail(MLB_E_INVAL, "workspace too small or not 256-byte aligned");
    mlb_grid* g = new (std::nothrow) mlb_grid();
    if (!g) return fail(MLB_E_NOMEM, "grid");
    g->ctx = c;
    g->p = *p;
    g->ld = ld;
    g->plane = align_up((size_t)ld * p->ny * sizeof(float), 256) / sizeof(float);
    if (ws) {
        g->base = (char*)ws;
    } else {
        hipError_t e = hipMalloc((void**)&g->base, need);
        if (e != hipSuccess) { delete g; return fail(MLB_E_NOMEM, std::string("hipMalloc: ") + hipGetErrorString(e)); }
        g->own = true;
    }
    g->stepc = (int64_t*)g->base;
    g->dres = (double*)(g->base + 64);
    float* f = (float*)(g->base + 256);
    g->eta[0] = f; g->eta[1] = f + g->plane;
    g->qx[0] = f + 2 * g->plane; g->qx[1] = f + 3 * g->plane;
    g->qy[0] = f + 4 * g->plane; g->qy[1] = f + 5 * g->plane;
    g->H = f + 6 * g->plane;
    g->e = 6.0 * p->nu / p->dx;   // Eq. (mlb-viscosity)
    g->dt = p->dx / g->e;
    c->live++;
    // default: flat bed one metre below the still-water level
    std::vector<double> zb((size_t)p->nx * p->ny, p->zeta_ref - 1.0);
    mlb_status s = mlb_set_bathymetry(g, zb.data(), p->nx);
    if (s != MLB_OK) { mlb_grid_destroy(g); return s; }
    *out = g;
    return MLB_OK;
}

mlb_status mlb_grid_destroy(mlb_grid* g)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    if (g->elab_refs) return fail(MLB_E_STATE, "an eLABSWE baseline still uses the grid");
    (void)hipSetDevice(g->ctx->device);
    (void)hipStreamSynchronize(g->ctx->stream);
    g->plan.release();
    if (g->own) (void)hipFree(g->base);
    if (g->dmask) (void)hipFree(g->dmask);
    if (g->dcoef) (void)hipFree(g->dcoef);
    if (g->etal) (void)hipFree(g->etal);
    g->ctx->live--;
    delete g;
    return MLB_OK;
}

mlb_status mlb_set_bathymetry(mlb_grid* g, const double* zb, int64_t ld)
{
    GRID_OK(g);
    if (!zb || ld < g->p.nx) return fail(MLB_E_INVAL, "zb is NULL or ld < nx");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    const int nx = g->p.nx, ny = g->p.ny;
    g->Hf.assign((size_t)g->ld * ny, 1.0f);
    g->Hd.assign((size_t)g->ld * ny, 1.0);
    double hmax = 0;
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const double Hd = g->p.zeta_ref - zb[(size_t)j * ld + i];
            if (!(Hd > 0)) return fail(MLB_E_INVAL, "still-water depth must be positive everywhere");
            const float Hs = (float)Hd;
            g->Hf[(size_t)j * g->ld + i] = Hs;
            g->Hd[(size_t)j * g->ld + i] = Hd;
            hmax = std::max(hmax, Hd);
        }
    if (g->p.g * hmax > g->e * g->e)
        return fail(MLB_E_UNSTABLE, "g * H_max > e^2: choose a larger nu (e = 6 nu / dx)");
    g->sumH = water_depth_sum(g);
    g->Hmax = hmax;
    CHK(implicit_coeffs(g));
    HIPCHK(hipMemcpyAsync(g->H, g->Hf.data(), g->Hf.size() * sizeof(float), hipMemcpyHostToDevice,
                          g->ctx->stream));
    CHK(upload_host_state(g, nullptr, nullptr, nullptr, nx));
    g->cur = 0;
    g->dirty = true;
    g->diag_fresh = false;
    return set_step(g, 0);
}

mlb_status mlb_set_wind(mlb_grid* g, double uwx, double uwy)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    const double s = std::sqrt(uwx * uwx + uwy * uwy);  // Eq. (wind_u-stress)
    return mlb_set_wind_stress(g, g->p.rho_air * g->p.c_w * uwx * s / g->p.rho_w,
                               g->p.rho_air * g->p.c_w * uwy * s / g->p.rho_w);
}

mlb_status mlb_set_wind_stress(mlb_grid* g, double tx, double ty)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    if (!std::isfinite(tx) || !std::isfinite(ty)) return fail(MLB_E_INVAL, "non-finite stress");
    g->tx = tx; g->ty = ty; g->dirty = true;
    return MLB_OK;
}

mlb_status mlb_set_chezy(mlb_grid* g, double cz)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    g->cb = cz > 0 ? g->p.g / (cz * cz) : 0.0;  // Eq. (bed-stress)
    g->dirty = true;
    return MLB_OK;
}

mlb_status mlb_set_edge_depth(mlb_grid* g, int edge, double h_mean, double amp, double period, double phase)
{
    if (!g || edge < 0 || edge > 3) return fail(MLB_E_INVAL, "bad grid or edge");
    if (g->p.edge[edge] != MLB_EDGE_DEPTH) return fail(MLB_E_INVAL, "edge is not a DEPTH edge");
    g->bc_hmean[edge] = h_mean; g->bc_amp[edge] = amp;
    g->bc_om[edge] = period > 0 ? 2.0 * M_PI / period : 0.0;
    g->bc_phase[edge] = phase;
    g->dirty = true;
    return MLB_OK;
}

mlb_status mlb_set_edge_discharge(mlb_grid* g, int edge, double qx, double qy)
{
    if (!g || edge < 0 || edge > 3) return fail(MLB_E_INVAL, "bad grid or edge");
    if (g->p.edge[edge] != MLB_EDGE_DISCHARGE) return fail(MLB_E_INVAL, "edge is not a DISCHARGE edge");
    g->bc_qx[edge] = qx; g->bc_qy[edge] = qy;
    g->dirty = true;
    return MLB_OK;
}

mlb_status mlb_plan_tiles(const mlb_params* p, const uint8_t* kind, int64_t kind_ld, int32_t tile_rows,
                          int32_t tblock, int32_t* tiles, int64_t capacity, int64_t* count)
{
    CHK(validate_params(p));
    if (!count || (capacity > 0 && !tiles)) return fail(MLB_E_INVAL, "count or tiles is NULL");
    if (tile_rows < 4 || tile_rows > 4096) return fail(MLB_E_INVAL, "tile_rows out of range");
    if (tblock != 1 && tblock != 2) return fail(MLB_E_INVAL, "tblock must be 1 or 2");
    if (kind && kind_ld < p->nx) return fail(MLB_E_INVAL, "kind_ld < nx");
    // a host-only grid: the tile builder reads the shape, edges and kinds
    mlb_grid g;
    g.p = *p;
    (void)field_bytes(p, &g.ld);
    if (kind) {
        g.hmask.assign((size_t)g.ld * p->ny, (uint8_t)NODE_FLUID);
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                const uint8_t k = kind[(size_t)j * kind_ld + i];
                if (k > NODE_SOLID) return fail(MLB_E_INVAL, "node kind must be FLUID, WALL or SOLID");
                g.hmask[(size_t)j * g.ld + i] = k;
            }
    }
    std::vector<TileDev> t;
    make_tiles(&g, 0, tile_rows, t, tblock == 2 ? kStripOut2 : kStripOut);
    *count = (int64_t)t.size();
    for (int64_t i = 0; i < std::min<int64_t>(capacity, (int64_t)t.size()); ++i) {
        int32_t* o = tiles + 6 * i;
        o[0] = t[i].x0; o[1] = t[i].y0; o[2] = t[i].rows; o[3] = t[i].xo; o[4] = t[i].yo; o[5] = t[i].flags;
    }
    return MLB_OK;
}

mlb_status mlb_plan_workqueue(const mlb_params* p, const uint8_t* kind, int64_t kind_ld, int32_t tile_rows,
                              int32_t tblock, int32_t* off, int64_t off_capacity, int32_t* nbr,
                              int64_t nbr_capacity, int64_t* ntiles, int64_t* nnbr)
{
    CHK(validate_params(p));
    if (!ntiles || !nnbr || (off_capacity > 0 && !off) || (nbr_capacity > 0 && !nbr))
        return fail(MLB_E_INVAL, "a count or list pointer is NULL");
    if (tile_rows < 4 || tile_rows > 4096) return fail(MLB_E_INVAL, "tile_rows out of range");
    if (tblock != 1 && tblock != 2) return fail(MLB_E_INVAL, "tblock must be 1 or 2");
    if (kind && kind_ld < p->nx) return fail(MLB_E_INVAL, "kind_ld < nx");
    mlb_grid g;
    g.p = *p;
    (void)field_bytes(p, &g.ld);
    if (kind) {
        g.hmask.assign((size_t)g.ld * p->ny, (uint8_t)NODE_FLUID);
        for (int j = 0; j < p->ny; ++j)
            for (int i = 0; i < p->nx; ++i) {
                const uint8_t k = kind[(size_t)j * kind_ld + i];
                if (k > NODE_SOLID) return fail(MLB_E_INVAL, "node kind must be FLUID, WALL or SOLID");
                g.hmask[(size_t)j * g.ld + i] = k;
            }
    }
    std::vector<TileDev> t;
    make_tiles(&g, 0, tile_rows, t, tblock == 2 ? kStripOut2 : kStripOut);
    std::vector<BasinDev> hb(1, make_basin(&g, 0));
    std::vector<int32_t> o, n;
    if (!wq_dependencies(hb, t, tblock, o, n))
        return fail(MLB_E_STATE, "a tile depends on more than 64 tiles: work-queue launches are not used");
    *ntiles = (int64_t)t.size();
    *nnbr = (int64_t)n.size();
    for (int64_t i = 0; i < std::min<int64_t>(off_capacity, (int64_t)o.size()); ++i) off[i] = o[i];
    for (int64_t i = 0; i < std::min<int64_t>(nbr_capacity, (int64_t)n.size()); ++i) nbr[i] = n[i];
    return MLB_OK;
}

mlb_status mlb_set_mask(mlb_grid* g, const uint8_t* kind, int64_t ld)
{
    GRID_OK(g);
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    const int nx = g->p.nx, ny = g->p.ny;
    if (!kind) {
        if (g->dmask) (void)hipFree(g->dmask);
        g->dmask = nullptr;
        g->hmask.clear();
    } else {
        if (ld < nx) return fail(MLB_E_INVAL, "ld < nx");
        std::vector<uint8_t> m((size_t)g->ld * ny, (uint8_t)NODE_FLUID);
        int64_t solid = 0;
        const int reach = g->p.extrap_order;
        for (int j = 0; j < ny; ++j)
            for (int i = 0; i < nx; ++i) {
                const uint8_t k = kind[(size_t)j * ld + i];
                if (k > NODE_SOLID) return fail(MLB_E_INVAL, "node kind must be FLUID, WALL or SOLID");
                m[(size_t)j * g->ld + i] = k;
                if (k == NODE_FLUID) continue;
                solid += k == NODE_SOLID;
                const int dist[4] = {i, nx - 1 - i, j, ny - 1 - j};
                for (int ed = 0; ed < 4; ++ed)
                    if (is_open(g->p.edge[ed]) && dist[ed] <= reach)
                        return fail(MLB_E_INVAL, "nodes an open edge extrapolates from must be FLUID");
            }
        if (solid == (int64_t)nx * ny) return fail(MLB_E_INVAL, "every node is SOLID");
        if (!g->dmask) HIPCHK(hipMalloc((void**)&g->dmask, m.size()));
        HIPCHK(hipMemcpyAsync(g->dmask, m.data(), m.size(), hipMemcpyHostToDevice, g->ctx->stream));
        // SOLID nodes are never written: both buffers must hold their values
        const size_t bytes = g->plane * sizeof(float);
        const int o = g->cur ^ 1;
        HIPCHK(hipMemcpyAsync(g->eta[o], g->eta[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qx[o], g->qx[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qy[o], g->qy[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        if (g->etal)
            HIPCHK(hipMemcpyAsync(g->etal + o * g->plane, g->etal + g->cur * g->plane, bytes, hipMemcpyDeviceToDevice,
                                  g->ctx->stream));
        HIPCHK(hipStreamSynchronize(g->ctx->stream));
        g->hmask.swap(m);
    }
    g->diag_fresh = false;   // the water (and so the sums) changed
    g->sumH = water_depth_sum(g);
    CHK(implicit_coeffs(g));
    g->stale_plan = true;
    return MLB_OK;
}

mlb_status mlb_set_surface(mlb_grid* g, int32_t mode)
{
    GRID_OK(g);
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    if (mode != MLB_SURFACE_FP32 && mode != MLB_SURFACE_COMPENSATED) return fail(MLB_E_INVAL, "unknown surface mode");
    const bool on = mode == MLB_SURFACE_COMPENSATED;
    if (on != (g->etal != nullptr)) {
        // the current state into the second buffer set (the next residual is 0)
        const size_t bytes = g->plane * sizeof(float);
        const int o = g->cur ^ 1;
        HIPCHK(hipMemcpyAsync(g->eta[o], g->eta[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qx[o], g->qx[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpyAsync(g->qy[o], g->qy[g->cur], bytes, hipMemcpyDeviceToDevice, g->ctx->stream));
        g->diag_fresh = false;
    }
    if (on && !g->etal) {
        HIPCHK(hipMalloc((void**)&g->etal, 2 * g->plane * sizeof(float)));
        HIPCHK(hipMemsetAsync(g->etal, 0, 2 * g->plane * sizeof(float), g->ctx->stream));
        HIPCHK(hipStreamSynchronize(g->ctx->stream));
        g->stale_plan = true;
    } else if (!on && g->etal) {
        HIPCHK(hipStreamSynchronize(g->ctx->stream));
        (void)hipFree(g->etal);
        g->etal = nullptr;
        g->stale_plan = true;
    }
    return MLB_OK;
}

mlb_status mlb_set_hbar(mlb_grid* g, int32_t mode)
{
    GRID_OK(g);
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    if (mode != MLB_HBAR_SEMI_IMPLICIT && mode != MLB_HBAR_IMPLICIT) return fail(MLB_E_INVAL, "unknown link-depth form");
    const int old = g->hbar;
    g->hbar = mode;
    mlb_status st = implicit_coeffs(g);
    if (st != MLB_OK) { g->hbar = old; return st; }
    if (mode != old) g->stale_plan = true;
    return MLB_OK;
}

mlb_status mlb_set_state(mlb_grid* g, const double* h, const double* hu, const double* hv, int64_t ld,
                         int64_t step0)
{
    GRID_OK(g);
    if (!h || ld < g->p.nx || step0 < 0) return fail(MLB_E_INVAL, "h is NULL, ld < nx or step0 < 0");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    CHK(upload_host_state(g, h, hu, hv, ld));
    g->diag_fresh = false;
    return set_step(g, step0);
}

mlb_status mlb_set_state_device(mlb_grid* g, const float* eta, const float* qx, const float* qy)
{
    GRID_OK(g);
    if (!eta || !qx || !qy) return fail(MLB_E_INVAL, "NULL device pointer");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    const size_t w = (size_t)g->p.nx * sizeof(float), pitch = (size_t)g->ld * sizeof(float);
    for (int k = 0; k < 2; ++k) {
        HIPCHK(hipMemcpy2DAsync(g->eta[k], pitch, eta, w, w, g->p.ny, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpy2DAsync(g->qx[k], pitch, qx, w, w, g->p.ny, hipMemcpyDeviceToDevice, g->ctx->stream));
        HIPCHK(hipMemcpy2DAsync(g->qy[k], pitch, qy, w, w, g->p.ny, hipMemcpyDeviceToDevice, g->ctx->stream));
    }
    if (g->etal) HIPCHK(hipMemsetAsync(g->etal, 0, 2 * g->plane * sizeof(float), g->ctx->stream));
    g->diag_fresh = false;
    return MLB_OK;
}

mlb_status mlb_get_state(mlb_grid* g, double* h, double* hu, double* hv, int64_t ld)
{
    GRID_OK(g);
    if (ld < g->p.nx) return fail(MLB_E_INVAL, "ld < nx");
    const int nx = g->p.nx, ny = g->p.ny;
    const size_t n = (size_t)g->ld * ny;
    std::unique_ptr<float[]> e(new (std::nothrow) float[n]), a(new (std::nothrow) float[n]),
        b(new (std::nothrow) float[n]);
    std::unique_ptr<float[]> el(g->etal ? new (std::nothrow) float[n] : nullptr);
    if (!e || !a || !b || (g->etal && !el)) return fail(MLB_E_NOMEM, "host staging of the state");
    const size_t bytes = n * sizeof(float);
    HIPCHK(hipMemcpyAsync(e.get(), g->eta[g->cur], bytes, hipMemcpyDeviceToHost, g->ctx->stream));
    HIPCHK(hipMemcpyAsync(a.get(), g->qx[g->cur], bytes, hipMemcpyDeviceToHost, g->ctx->stream));
    HIPCHK(hipMemcpyAsync(b.get(), g->qy[g->cur], bytes, hipMemcpyDeviceToHost, g->ctx->stream));
    if (g->etal)
        HIPCHK(hipMemcpyAsync(el.get(), g->etal + g->cur * g->plane, bytes, hipMemcpyDeviceToHost, g->ctx->stream));
    HIPCHK(hipStreamSynchronize(g->ctx->stream));
    CHK(check_abort(g->ctx, g->plan));
    for_rows(ny, (size_t)nx * ny, [&](int j0, int j1) {
        for (int j = j0; j < j1; ++j)
            for (int i = 0; i < nx; ++i) {
                const size_t s = (size_t)j * g->ld + i, d = (size_t)j * ld + i;
                if (h) h[d] = g->Hd[s] + (double)e[s] + (g->etal ? (double)el[s] : 0.0);
                if (hu) hu[d] = a[s];
                if (hv) hv[d] = b[s];
            }
    });
    return MLB_OK;
}

mlb_status mlb_get_state_device(mlb_grid* g, float* eta, float* qx, float* qy, float* H)
{
    GRID_OK(g);
    CHK(check_abort(g->ctx, g->plan));   // waits only after a persistent launch
    const size_t w = (size_t)g->p.nx * sizeof(float), pitch = (size_t)g->ld * sizeof(float);
    const int ny = g->p.ny;
    if (eta) HIPCHK(hipMemcpy2DAsync(eta, w, g->eta[g->cur], pitch, w, ny, hipMemcpyDeviceToDevice, g->ctx->stream));
    if (qx) HIPCHK(hipMemcpy2DAsync(qx, w, g->qx[g->cur], pitch, w, ny, hipMemcpyDeviceToDevice, g->ctx->stream));
    if (qy) HIPCHK(hipMemcpy2DAsync(qy, w, g->qy[g->cur], pitch, w, ny, hipMemcpyDeviceToDevice, g->ctx->stream));
    if (H) HIPCHK(hipMemcpy2DAsync(H, w, g->H, pitch, w, ny, hipMemcpyDeviceToDevice, g->ctx->stream));
    return MLB_OK;
}

mlb_status mlb_get_exec_opts(const mlb_grid* g, mlb_exec_opts* o)
{
    if (!g || !o) return fail(MLB_E_INVAL, "NULL argument");
    *o = g->opts;
    return MLB_OK;
}

static mlb_status check_opts(const mlb_exec_opts* o)
{
    if (!o) return fail(MLB_E_INVAL, "opts is NULL");
    if (o->tile_rows < 4 || o->tile_rows > 4096) return fail(MLB_E_INVAL, "tile_rows out of range");
    if (o->tblock != 1 && o->tblock != 2) return fail(MLB_E_INVAL, "tblock must be 1 or 2");
    if (o->blocks_per_cu < 0 || o->blocks_per_cu > 8) return fail(MLB_E_INVAL, "blocks_per_cu must be 0..8");
    if (o->use_graph && (o->graph_chunk < 2 || o->graph_chunk > 100000))
        return fail(MLB_E_INVAL, "graph_chunk out of range");
    if (o->persistent < 0 || o->persistent > 2) return fail(MLB_E_INVAL, "persistent must be 0, 1 or 2");
    return MLB_OK;
}

mlb_status mlb_set_exec_opts(mlb_grid* g, const mlb_exec_opts* o)
{
    if (!g) return fail(MLB_E_INVAL, "grid is NULL");
    CHK(check_opts(o));
    if (o->tile_rows != g->opts.tile_rows || o->tblock != g->opts.tblock) g->stale_plan = true;
    g->opts = *o;
    return MLB_OK;
}

// n steps in `launches` launches: each launch swaps the buffers once
static void advance_grid(mlb_grid* g, int64_t n, int64_t launches)
{
    g->step += n;
    if (launches & 1) g->cur ^= 1;
}

mlb_status mlb_step(mlb_grid* g, int64_t n)
{
    GRID_OK(g);
    if (n < 0) return fail(MLB_E_INVAL, "nsteps < 0");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    if (n == 0) return MLB_OK;
    CHK(grid_plan(g));
    mlb_ctx* c = g->ctx;
    CHK(peek_abort(c, g->plan));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    int64_t nl = 0;
    CHK(enqueue_steps(c, g->plan, g->opts, n, true, &nl));
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    c->timed = true;
    advance_grid(g, n, nl);
    g->diag_fresh = true;   // the closing checked pass filled the result slot
    return MLB_OK;
}

mlb_status mlb_diag(mlb_grid* g, mlb_diag_t* out)
{
    GRID_OK(g);
    if (!out) return fail(MLB_E_INVAL, "out is NULL");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    CHK(grid_plan(g));
    Plan& P = g->plan;
    mlb_ctx* c = g->ctx;
    if (!g->diag_fresh) {
        // the fields were set since the last checked pass: reduce the state
        // (both buffers hold it, so the residual is 0)
        HIPCHK(launch_reduce_state(P.db, P.dt, (int)P.ht.size(), P.parity, P.dpart, c->stream));
        HIPCHK(launch_finalize(P.db, 1, P.dpart, P.dout, 1, c->stream));
        g->diag_fresh = true;
    }
    HIPCHK(hipMemcpyAsync(P.hout, g->dres, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(hipStreamSynchronize(c->stream));
    CHK(check_abort(c, P));
    fill_diag(g, P.hout, out);
    return MLB_OK;
}

mlb_status mlb_run_steady(mlb_grid* g, double tol, int64_t max_steps, int32_t check_every, mlb_diag_t* out)
{
    GRID_OK(g);
    if (check_every < 1 || max_steps < 1 || !(tol >= 0)) return fail(MLB_E_INVAL, "bad tol / max_steps / check_every");
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    CHK(grid_plan(g));
    mlb_ctx* c = g->ctx;
    const int64_t start = g->step;
    mlb_diag_t d{};
    double best = INFINITY;
    int since = 0;
    while (g->step - start < max_steps) {
        const int64_t n = std::min<int64_t>(check_every, max_steps - (g->step - start));
        int64_t nl = 0;
        CHK(enqueue_steps(c, g->plan, g->opts, n, true, &nl));
        advance_grid(g, n, nl);
        g->diag_fresh = true;
        CHK(read_diag(c, g->plan));
        fill_diag(g, g->plan.hout, &d);
        if (out) *out = d;
        if (d.nonfinite) return fail(MLB_E_NONFINITE, "non-finite value or dry node");
        if (d.residual <= tol) return MLB_OK;
        if (d.residual < best) { best = d.residual; since = 0; }
        else if (c->stall_checks > 0 && best <= kStallBand * tol && ++since >= c->stall_checks)
            return fail(MLB_E_STALLED, "residual stalled");
    }
    return fail(MLB_E_NOTCONVERGED, "max_steps reached");
}

mlb_status mlb_last_step_ms(mlb_ctx* c, double* ms)
{
    if (!c || !ms) return fail(MLB_E_INVAL, "NULL argument");
    if (!c->timed) return fail(MLB_E_STATE, "no timed step yet");
    CHK(check_stream(c));
    HIPCHK(hipEventSynchronize(c->ev1));
    float f = 0;
    HIPCHK(hipEventElapsedTime(&f, c->ev0, c->ev1));
    *ms = f;
    return MLB_OK;
}

mlb_status mlb_last_pass_ms(mlb_ctx* c, double* ms, int64_t* passes, int32_t* steps_per_pass)
{
    if (!c || !ms) return fail(MLB_E_INVAL, "NULL argument");
    if (!c->timed) return fail(MLB_E_STATE, "no timed step yet");
    if (c->bulk_passes < 1) return fail(MLB_E_STATE, "the last call had no passes besides its checked one");
    CHK(check_stream(c));
    HIPCHK(hipEventSynchronize(c->ev3));
    float f = 0;
    HIPCHK(hipEventElapsedTime(&f, c->ev2, c->ev3));
    *ms = f / (double)c->bulk_passes;
    if (passes) *passes = c->bulk_passes;
    if (steps_per_pass) *steps_per_pass = c->bulk_kind;
    return MLB_OK;
}

mlb_status mlb_copy_probe(mlb_ctx* c, size_t bytes, int32_t reps, double* gbps)
{
    if (!c || !gbps || reps < 1 || bytes < 4096 || (bytes & 15)) return fail(MLB_E_INVAL, "bad copy probe arguments");
    CHK(check_stream(c));
    void *a = nullptr, *b = nullptr;
    HIPCHK(hipMalloc(&a, bytes));
    hipError_t e = hipMalloc(&b, bytes);
    if (e != hipSuccess) { (void)hipFree(a); return fail(MLB_E_NOMEM, hipGetErrorString(e)); }
    const int nblocks = c->ncu * 8;
    e = hipMemsetAsync(a, 0, bytes, c->stream);
    if (e == hipSuccess) e = launch_copy_probe(a, b, bytes, nblocks, c->stream);  // warm-up
    if (e == hipSuccess) e = hipEventRecord(c->ev0, c->stream);
    for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch_copy_probe(a, b, bytes, nblocks, c->stream);
    if (e == hipSuccess) e = hipEventRecord(c->ev1, c->stream);
    if (e == hipSuccess) e = hipEventSynchronize(c->ev1);
    float ms = 0;
    if (e == hipSuccess) e = hipEventElapsedTime(&ms, c->ev0, c->ev1);
    (void)hipFree(a);
    (void)hipFree(b);
    if (e != hipSuccess) return fail(MLB_E_DEVICE, hipGetErrorString(e));
    *gbps = 2.0 * (double)bytes * reps / (ms * 1e-3) / 1e9;
    return MLB_OK;
}

// ------------------------------------------------------------------ batches
static mlb_status batch_plan(mlb_batch* b)
{
    if (!b->stale_plan && b->plan.built) return MLB_OK;
    b->plan.release();
    const int n = (int)b->grids.size();
    std::vector<int> order(n);
    for (int i = 0; i < n; ++i) order[i] = i;
    // largest basins first so their tiles enter the queue first
    std::stable_sort(order.begin(), order.end(), [&](int a, int c) {
        return (int64_t)b->grids[a]->p.nx * b->grids[a]->p.ny > (int64_t)b->grids[c]->p.nx * b->grids[c]->p.ny;
    });
    b->plan.hb.assign(n, BasinDev{});
    b->plan.ht.clear();
    b->plan.ht2.clear();
    b->plan.parity = 0;
    bool masked = false;
    for (auto* g : b->grids) masked |= g->dmask != nullptr;
    const bool implicit = b->grids[0]->hbar == MLB_HBAR_IMPLICIT;   // shared by every grid
    const bool comp = b->grids[0]->etal != nullptr;                  // likewise
    for (int k = 0; k < n; ++k) {
        const int i = order[k];
        mlb_grid* g = b->grids[i];
        BasinDev d = make_basin(g, g->cur);
        d.first_tile = (int)b->plan.ht.size();
        make_tiles(g, i, b->opts.tile_rows, b->plan.ht, kStripOut);
        d.ntiles = (int)b->plan.ht.size() - d.first_tile;
        d.first_tile2 = (int)b->plan.ht2.size();
        if (b->opts.tblock == 2 && !comp)
            make_tiles(g, i, b->opts.tile_rows, b->plan.ht2, kStripOut2);
        d.ntiles2 = (int)b->plan.ht2.size() - d.first_tile2;
        b->plan.hb[i] = d;
    }
    // (Putting all basins' costly two-step tiles ahead of all others, across
    // basins, was measured 6 % slower on the 512-basin ensemble than ordering
    // within each basin: the basins' tiles then no longer run together.)
    b->plan.masked = masked;
    b->plan.implicit = implicit;
    b->plan.comp = comp;
    b->plan.closed = true;
    for (auto* g : b->grids) b->plan.closed = b->plan.closed && !has_open_edge(g);
    CHK(plan_alloc(b->ctx, b->plan));
    b->stale_plan = false;
    return MLB_OK;
}

mlb_status mlb_batch_create(mlb_ctx* c, mlb_grid* const* grids, int32_t n, mlb_batch** out)
{
    if (!c || !grids || n < 1 || !out) return fail(MLB_E_INVAL, "bad batch arguments");
    *out = nullptr;
    CHK(check_stream(c));
    for (int i = 0; i < n; ++i) {
        if (!grids[i] || grids[i]->ctx != c) return fail(MLB_E_INVAL, "grid missing or from another context");
        if (grids[i]->batch) return fail(MLB_E_STATE, "grid already in a batch");
        if (grids[i]->hbar != grids[0]->hbar)
            return fail(MLB_E_INVAL, "the grids of a batch must share the link-depth form");
        if ((grids[i]->etal != nullptr) != (grids[0]->etal != nullptr))
            return fail(MLB_E_INVAL, "the grids of a batch must share the surface precision");
        for (int k = 0; k < i; ++k)
            if (grids[k] == grids[i]) return fail(MLB_E_INVAL, "grid listed twice");
    }
    mlb_batch* b = new (std::nothrow) mlb_batch();
    if (!b) return fail(MLB_E_NOMEM, "batch");
    b->ctx = c;
    b->grids.assign(grids, grids + n);
    b->opts = grids[0]->opts;
    HIPCHK(hipStreamSynchronize(c->stream));
    mlb_status s = batch_plan(b);
    if (s != MLB_OK) { b->plan.release(); delete b; return s; }
    for (auto* g : b->grids) g->batch = b;
    c->live++;
    *out = b;
    return MLB_OK;
}

mlb_status mlb_batch_set_exec_opts(mlb_batch* b, const mlb_exec_opts* o)
{
    if (!b) return fail(MLB_E_INVAL, "batch is NULL");
    CHK(check_opts(o));
    if (o->tile_rows != b->opts.tile_rows || o->tblock != b->opts.tblock) {
        // rebuild with the current buffers as the starting parity
        b->stale_plan = true;
    }
    b->opts = *o;
    return MLB_OK;
}

mlb_status mlb_batch_step(mlb_batch* b, int64_t n)
{
    if (!b) return fail(MLB_E_INVAL, "batch is NULL");
    if (n < 0) return fail(MLB_E_INVAL, "nsteps < 0");
    CHK(check_stream(b->ctx));
    if (n == 0) return MLB_OK;
    CHK(batch_plan(b));
    mlb_ctx* c = b->ctx;
    CHK(peek_abort(c, b->plan));
    HIPCHK(hipEventRecord(c->ev0, c->stream));
    int64_t nl = 0;
    CHK(enqueue_steps(c, b->plan, b->opts, n, true, &nl));
    HIPCHK(hipEventRecord(c->ev1, c->stream));
    c->timed = true;
    for (auto* g : b->grids) { advance_grid(g, n, nl); g->diag_fresh = true; }
    return MLB_OK;
}

mlb_status mlb_batch_run_steady(mlb_batch* b, double tol, int64_t max_steps, int32_t check_every,
                                mlb_diag_t* per)
{
    if (!b) return fail(MLB_E_INVAL, "batch is NULL");
    if (check_every < 1 || max_steps < 1 || !(tol >= 0)) return fail(MLB_E_INVAL, "bad tol / max_steps / check_every");
    CHK(check_stream(b->ctx));
    CHK(batch_plan(b));
    mlb_ctx* c = b->ctx;
    int64_t done = 0;
    const int n = (int)b->grids.size();
    while (done < max_steps) {
        const int64_t k = std::min<int64_t>(check_every, max_steps - done);
        int64_t nl = 0;
        CHK(enqueue_steps(c, b->plan, b->opts, k, true, &nl));
        for (auto* g : b->grids) { advance_grid(g, k, nl); g->diag_fresh = true; }
        done += k;
        CHK(read_diag(c, b->plan));
        bool all = true, bad = false;
        for (int i = 0; i < n; ++i) {
            mlb_diag_t d{};
            fill_diag(b->grids[i], b->plan.hout + 8 * i, &d);
            if (per) per[i] = d;
            bad |= d.nonfinite != 0;
            all &= d.residual <= tol;
        }
        if (bad) return fail(MLB_E_NONFINITE, "non-finite value or dry node in a basin");
        if (all) return MLB_OK;
    }
    return fail(MLB_E_NOTCONVERGED, "max_steps reached");
}

mlb_status mlb_batch_destroy(mlb_batch* b)
{
    if (!b) return fail(MLB_E_INVAL, "batch is NULL");
    (void)hipSetDevice(b->ctx->device);
    (void)hipStreamSynchronize(b->ctx->stream);
    b->plan.release();
    for (auto* g : b->grids) {
        g->batch = nullptr;
        g->dirty = true;   // the grid's own plan must re-derive its buffer parity
    }
    b->ctx->live--;
    delete b;
    return MLB_OK;
}

}  // extern "C"

// ------------------------------------------------------------------ autotuner
namespace {

// One-step tiles cost least at 3k rows, two-step interior tiles at 3k + 2
// (their walk ends with two rows of the second stage alone).  The shortest
// tiles serve small grids, where a wave's serial row walk, not bandwidth,
// sets the time of a pass.
const int kTuneRows[] = {4, 6, 9, 12, 15, 21, 27, 33, 45};
const int kTuneRows2[] = {4, 5, 8, 11, 14, 17, 20, 23, 26, 32, 44};
const int kTuneCaps[] = {0, 2, 3, 4, 5};
const int kTuneBlocks[] = {1, 2};

// Device copies of the current fields of some grids, to restore after tuning.
struct Saved {
    std::vector<float*> buf;
    std::vector<int64_t> step;
    void release() { for (float* p : buf) (void)hipFree(p); buf.clear(); }
};

mlb_status save_states(mlb_ctx* c, const std::vector<mlb_grid*>& gs, Saved& sv)
{
    for (mlb_grid* g : gs) {
        float* p = nullptr;
        HIPCHK(hipMalloc(&p, 4 * g->plane * sizeof(float)));
        sv.buf.push_back(p);
        sv.step.push_back(g->step);
        if (g->etal)
            HIPCHK(hipMemcpyAsync(p + 3 * g->plane, g->etal + g->cur * g->plane, g->plane * sizeof(float),
                                  hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(p, g->eta[g->cur], g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(p + g->plane, g->qx[g->cur], g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(hipMemcpyAsync(p + 2 * g->plane, g->qy[g->cur], g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
    }
    return MLB_OK;
}

mlb_status restore_states(mlb_ctx* c, const std::vector<mlb_grid*>& gs, Saved& sv)
{
    for (size_t i = 0; i < gs.size(); ++i) {
        mlb_grid* g = gs[i];
        const float* p = sv.buf[i];
        for (int k = 0; k < 2; ++k) {  // both buffers: the next residual is 0
            HIPCHK(hipMemcpyAsync(g->eta[k], p, g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(g->qx[k], p + g->plane, g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
            HIPCHK(hipMemcpyAsync(g->qy[k], p + 2 * g->plane, g->plane * sizeof(float), hipMemcpyDeviceToDevice, c->stream));
            if (g->etal)
                HIPCHK(hipMemcpyAsync(g->etal + k * g->plane, p + 3 * g->plane, g->plane * sizeof(float),
                                      hipMemcpyDeviceToDevice, c->stream));
        }
        CHK(set_step(g, sv.step[i]));
        g->diag_fresh = false;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    return MLB_OK;
}

bool cache_lookup(const char* path, const std::string& key, mlb_exec_opts* o)
{
    if (!path) return false;
    FILE* f = std::fopen(path, "r");
    if (!f) return false;
    char k[256];
    int tr = 0, bc = 0, tb = 1, ps = 0;
    double us = 0;
    bool hit = false;
    while (std::fscanf(f, "%255s %d %d %d %d %lf", k, &tr, &bc, &tb, &ps, &us) == 6)
        if (key == k) { o->tile_rows = tr; o->blocks_per_cu = bc; o->tblock = tb; o->persistent = ps; hit = true; }
    std::fclose(f);
    return hit;
}

void cache_store(const char* path, const std::string& key, const mlb_exec_opts& o, double us)
{
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %d %d %.3f\n", key.c_str(), o.tile_rows, o.blocks_per_cu, o.tblock, o.persistent, us);
    std::fclose(f);
}

// Whether the tiles of these grids at (rows, tblock) fit on the device at once.
bool fits_persistent(mlb_ctx* c, const std::vector<mlb_grid*>& gs, int rows, int tb)
{
    int64_t tiles = 0;
    const int strip = tb == 2 ? kStripOut2 : kStripOut;
    bool masked = false;
    for (auto* g : gs) masked |= g->dmask != nullptr;
    for (auto* g : gs) {
        std::vector<TileDev> t;
        make_tiles(g, 0, rows, t, strip);
        tiles += (int64_t)t.size();
    }
    const int64_t nblk = (tiles + kBlock / kWave - 1) / (kBlock / kWave);
    return nblk <= persistent_capacity(tb, masked ? 1 : 0, c->ncu);
}

// Times `steps` steps of each candidate; `prepare` rebuilds the plan for the
// options and returns it.  Leaves *opts at the fastest candidate.
template <class Prepare>
mlb_status tune(mlb_ctx* c, mlb_exec_opts* opts, int steps, const std::vector<mlb_grid*>& gs,
                Prepare prepare, double* best_us)
{
    const mlb_exec_opts base = *opts;
    mlb_exec_opts best = base;
    double best_t = 1e300;
    const int n = std::max(2, steps & ~1);
    bool one = false;   // the compensated surface runs one step per pass
    for (auto* g : gs) one |= g->etal != nullptr;
    struct Cand { double us; mlb_exec_opts o; };
    std::vector<Cand> cands;
    int tried[3] = {0, 0, 0};
    double mode_best[3] = {1e300, 1e300, 1e300};
    for (int ps = 0; ps < 3; ++ps)
    for (int tb : kTuneBlocks)
    for (int tr : (tb == 2 ? std::vector<int>(std::begin(kTuneRows2), std::end(kTuneRows2))
                           : std::vector<int>(std::begin(kTuneRows), std::end(kTuneRows))))
        for (int cap : kTuneCaps) {
            // cooperative launches need every tile resident: no workgroup cap
            if (ps == 1 && (cap != 0 || !fits_persistent(c, gs, tr, tb))) continue;
            if (one && tb == 2) continue;
            // a persistent mode whose first two candidates take more than twice
            // the best ordinary launch is not timed further
            if (ps > 0 && tried[ps] >= 2 && mode_best[ps] > 2.0 * best_t) continue;
            mlb_exec_opts o = base;
            o.persistent = ps;
            o.tblock = tb;
            o.tile_rows = tr;
            o.blocks_per_cu = cap;
            o.use_graph = 1;
            o.graph_chunk = n;
            *opts = o;
            Plan* P = nullptr;
            CHK(prepare(o, &P));
            int64_t nl = 0;
            CHK(enqueue_steps(c, *P, o, n, false, &nl));  // capture + warm-up
            for (auto* g : gs) advance_grid(g, n, nl);
            float ms[3];
            for (int rep = 0; rep < 3; ++rep) {
                HIPCHK(hipEventRecord(c->ev0, c->stream));
                CHK(enqueue_steps(c, *P, o, n, false, &nl));
                HIPCHK(hipEventRecord(c->ev1, c->stream));
                HIPCHK(hipEventSynchronize(c->ev1));
                HIPCHK(hipEventElapsedTime(&ms[rep], c->ev0, c->ev1));
                for (auto* g : gs) advance_grid(g, n, nl);
            }
            ++tried[ps];
            // a persistent candidate whose barrier wait gave up did not run its
            // passes: never a candidate (the state is restored afterwards)
            if (check_abort(c, *P) != MLB_OK) continue;
            std::sort(ms, ms + 3);
            const double us = 1e3 * ms[1] / n;
            mode_best[ps] = std::min(mode_best[ps], us);
            cands.push_back({us, o});
            if (us < best_t) { best_t = us; best = o; }
        }
    // The fastest few again, over longer runs: runs of a few milliseconds
    // rank neighbouring options (tile heights, workgroup caps) within their
    // noise.  Median of five runs of at least 200 steps each.
    std::stable_sort(cands.begin(), cands.end(), [](const Cand& x, const Cand& y) { return x.us < y.us; });
    const int n2 = std::max(n, 200) & ~1;
    double best2 = 1e300;
    for (size_t k = 0; k < cands.size() && k < 4; ++k) {
        mlb_exec_opts o = cands[k].o;
        o.graph_chunk = n2;
        *opts = o;
        Plan* P = nullptr;
        CHK(prepare(o, &P));
        int64_t nl = 0;
        CHK(enqueue_steps(c, *P, o, n2, false, &nl));   // capture + warm-up
        for (auto* g : gs) advance_grid(g, n2, nl);
        float ms[5];
        for (int rep = 0; rep < 5; ++rep) {
            HIPCHK(hipEventRecord(c->ev0, c->stream));
            CHK(enqueue_steps(c, *P, o, n2, false, &nl));
            HIPCHK(hipEventRecord(c->ev1, c->stream));
            HIPCHK(hipEventSynchronize(c->ev1));
            HIPCHK(hipEventElapsedTime(&ms[rep], c->ev0, c->ev1));
            for (auto* g : gs) advance_grid(g, n2, nl);
        }
        if (check_abort(c, *P) != MLB_OK) continue;
        std::sort(ms, ms + 5);
        const double us = 1e3 * ms[2] / n2;
        if (us < best2) { best2 = us; best = cands[k].o; best_t = us; }
    }
    best.use_graph = base.use_graph;
    best.graph_chunk = base.graph_chunk;
    *opts = best;
    *best_us = best_t;
    return MLB_OK;
}

}  // namespace

extern "C" {

mlb_status mlb_autotune(mlb_grid* g, int32_t steps, const char* cache_path, mlb_exec_opts* best)
{
    GRID_OK(g);
    if (g->batch) return fail(MLB_E_STATE, "grid belongs to a live batch");
    if (steps < 2) return fail(MLB_E_INVAL, "steps must be >= 2");
    mlb_ctx* c = g->ctx;
    const std::string key = c->arch + "_g" + std::to_string(g->p.nx) + "x" + std::to_string(g->p.ny) +
                            (g->dmask ? "m" : "") + (g->hbar == MLB_HBAR_IMPLICIT ? "i" : "") +
                            (g->etal ? "c" : "");
    mlb_exec_opts o = g->opts;
    if (cache_lookup(cache_path, key, &o)) {
        CHK(mlb_set_exec_opts(g, &o));
        if (best) *best = g->opts;
        return MLB_OK;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    std::vector<mlb_grid*> gs{g};
    Saved sv;
    mlb_status st = save_states(c, gs, sv);
    double us = 0;
    if (st == MLB_OK)
        st = tune(c, &o, steps, gs, [&](const mlb_exec_opts& oo, Plan** P) -> mlb_status {
            if (oo.tile_rows != g->opts.tile_rows || oo.tblock != g->opts.tblock) g->stale_plan = true;
            g->opts = oo;
            CHK(grid_plan(g));
            *P = &g->plan;
            return MLB_OK;
        }, &us);
    mlb_status rs = st == MLB_OK || !sv.buf.empty() ? restore_states(c, gs, sv) : MLB_OK;
    sv.release();
    if (st != MLB_OK) return st;
    if (rs != MLB_OK) return rs;
    g->stale_plan = true;
    g->opts = o;
    cache_store(cache_path, key, o, us);
    if (best) *best = o;
    return MLB_OK;
}

mlb_status mlb_batch_autotune(mlb_batch* b, int32_t steps, const char* cache_path, mlb_exec_opts* best)
{
    if (!b) return fail(MLB_E_INVAL, "batch is NULL");
    if (steps < 2) return fail(MLB_E_INVAL, "steps must be >= 2");
    mlb_ctx* c = b->ctx;
    CHK(check_stream(c));
    int64_t nodes = 0;
    bool masked = false;
    for (auto* g : b->grids) { nodes += (int64_t)g->p.nx * g->p.ny; masked |= g->dmask != nullptr; }
    const std::string key = c->arch + "_b" + std::to_string(b->grids.size()) + "n" + std::to_string(nodes) +
                            (masked ? "m" : "") + (b->grids[0]->hbar == MLB_HBAR_IMPLICIT ? "i" : "") +
                            (b->grids[0]->etal ? "c" : "");
    mlb_exec_opts o = b->opts;
    if (cache_lookup(cache_path, key, &o)) {
        CHK(mlb_batch_set_exec_opts(b, &o));
        if (best) *best = b->opts;
        return MLB_OK;
    }
    HIPCHK(hipStreamSynchronize(c->stream));
    Saved sv;
    mlb_status st = save_states(c, b->grids, sv);
    double us = 0;
    if (st == MLB_OK)
        st = tune(c, &o, steps, b->grids, [&](const mlb_exec_opts& oo, Plan** P) -> mlb_status {
            if (oo.tile_rows != b->opts.tile_rows || oo.tblock != b->opts.tblock) b->stale_plan = true;
            b->opts = oo;
            CHK(batch_plan(b));
            *P = &b->plan;
            return MLB_OK;
        }, &us);
    mlb_status rs = !sv.buf.empty() ? restore_states(c, b->grids, sv) : MLB_OK;
    sv.release();
    if (st != MLB_OK) return st;
    if (rs != MLB_OK) return rs;
    b->stale_plan = true;  // re-derive buffer parities from the restored grids
    b->opts = o;
    cache_store(cache_path, key, o, us);
    if (best) *best = o;
    return MLB_OK;
}

}  // extern "C"
