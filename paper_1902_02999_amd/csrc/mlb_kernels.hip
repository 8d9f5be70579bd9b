// gfx950 kernels of the MacLABSWE streaming-only step (Zhou, arXiv 1902.02999).
//
// Arithmetic (per node x, upstream neighbours y_a = x - e_a dt, FP32):
//   The paper's update (Eqs. Mac.lb.3, Mac.lb.6, Mac.lb.7 with the centred
//   bed term of Eq. h-bar and the centred force of Eq. force-CS) is evaluated
//   in an algebraically identical increment form.  Splitting the equilibrium
//   of Eq. feq-full as f_a^eq = C_a g h^2 / (2 e^2) + A_a(h, q):
//     - the hydrostatic part of f_a^eq(y) and the bed term combine into
//       C_a g/(2e^2) (h_x + h_y)(eta_y - eta_x), with eta = h - H, so still
//       water gives exactly zero in any precision (well-balanced);
//     - the rest-particle equilibrium cancels the hydrostatic parts at x;
//     - the force is folded into the linear part of A_a as q~ = q + (dt/2) F
//       (C_a / e = lambda_a / (3e)), which carries the link-midpoint average;
//     - a bounced link (upstream outside a wall) takes A_abar(x) and no bed
//       or force term, i.e. the values of a virtual neighbour with eta_y = eta_x
//       and A_a(y) = A_abar(x).
//   With Out_a(n) = A_a built from q~(n), kk = 2K/(3e^2), K = q.u:
//     eta' = eta + sum_a Out_a(y_a) - kk + g/(2e^2) sum_a C_a P_a
//     q'   = (dt/2) F(x) + e sum_a e^_a Out_a(y_a) + g/(2e) sum_a C_a e^_a P_a
//   where P_a = (h_x + h_y)(eta_y - eta_x).
//
// Execution: each wave walks a strip of 62 output columns down a tile of rows
// (a column per lane, lanes 0 and 63 are the halo).  Per row it loads
// eta, qx, qy, H once (coalesced SoA rows), derives the node quantities once,
// and passes the ones its neighbours need across lanes with DPP wave shifts;
// a three-row register window gives the 8-neighbour gather.  One wave per
// tile; the tile list holds the largest basins first.
#include "mlb_internal.h"

// Build-time knob (results are bitwise independent of it):
//   MLB_NT_STORE  non-temporal stores of the new fields (written once per step)
#ifndef MLB_NT_STORE
#define MLB_NT_STORE 1
#endif

namespace mlb {

// ------------------------------------------------------------------ lanes
// DPP wave shifts; lanes without a source (lane 0 / lane 63) read 0
__device__ __forceinline__ float from_left(float v)  // lane i receives lane i-1
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x138 /* wave_shr:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ float from_right(float v)  // lane i receives lane i+1
{
    return __builtin_bit_cast(float, __builtin_amdgcn_mov_dpp(
        __builtin_bit_cast(int, v), 0x130 /* wave_shl:1 */, 0xf, 0xf, true));
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) double gdouble;

// ------------------------------------------------------------------ node arithmetic
struct Derived {
    float eta, h, kk, fpx, fpy;
    float o[9];            // o[a] = Out_a(node), a = 1..8
    float H, q0x, q0y;     // the node's stored H and old discharge
};

// Node quantities from the old state (Eqs. SWE-force, bed-stress, feq-full).
__device__ __forceinline__ void derive(const BasinDev& B, float eta, float qx, float qy, float H,
                                       Derived& d)
{
    const float h = H + eta;
    const float r = __builtin_amdgcn_rcpf(h);
    const float u = qx * r, v = qy * r;
    const float s = __builtin_amdgcn_sqrtf(__builtin_fmaf(u, u, v * v));
    const float fr = B.cfr * s;
    // (dt/2) F = (dt/2) [tau_w/rho - C_b u |u| + Omega (qy, -qx)]
    const float fpx = __builtin_fmaf(B.omh, qy, __builtin_fmaf(-fr, u, B.tpx));
    const float fpy = __builtin_fmaf(-B.omh, qx, __builtin_fmaf(-fr, v, B.tpy));
    const float tqx = qx + fpx, tqy = qy + fpy;
    const float pxx = qx * u, pyy = qy * v, pxy = qx * v;
    const float kq = pxx + pyy;
    const float lx = B.c3e * tqx, ly = B.c3e * tqy;
    const float qxx = B.c6 * __builtin_fmaf(2.0f, pxx, -pyy);
    const float qyy = B.c6 * __builtin_fmaf(2.0f, pyy, -pxx);
    const float qd = B.c12 * kq, rxy = B.c4 * pxy;
    const float qd1 = qd + rxy, qd2 = qd - rxy;
    const float ldp = 0.25f * (lx + ly), ldm = 0.25f * (lx - ly);
    d.o[0] = 0.0f;
    d.o[1] = qxx + lx;  d.o[5] = qxx - lx;
    d.o[3] = qyy + ly;  d.o[7] = qyy - ly;
    d.o[2] = qd1 + ldp; d.o[6] = qd1 - ldp;
    d.o[4] = qd2 - ldm; d.o[8] = qd2 + ldm;
    d.eta = eta; d.h = h; d.kk = B.ckk * kq; d.fpx = fpx; d.fpy = fpy;
    d.H = H; d.q0x = qx; d.q0y = qy;
}

// Eqs. Mac.lb.6 / Mac.lb.7 in increment form from the gathered neighbour
// equilibria oy[a] = Out_a(y_a) and link products P[a] = (h_x + h_y)(eta_y - eta_x).
__device__ __forceinline__ void update(const BasinDev& B, const Derived& x, const float* P,
                                       const float* oy, float& eta_n, float& qx_n, float& qy_n)
{
    const float so = ((oy[1] + oy[2]) + (oy[3] + oy[4])) + ((oy[5] + oy[6]) + (oy[7] + oy[8]));
    const float pa = (P[1] + P[3]) + (P[5] + P[7]);
    const float pd = (P[2] + P[4]) + (P[6] + P[8]);
    const float mp = __builtin_fmaf(B.cma, pa, B.cmd * pd);
    eta_n = x.eta + ((so - x.kk) + mp);
    const float o26 = oy[2] - oy[6], p26 = P[2] - P[6];
    const float mxo = (oy[1] - oy[5]) + (o26 + (oy[8] - oy[4]));
    const float myo = (oy[3] - oy[7]) + (o26 + (oy[4] - oy[8]));
    const float pxm = __builtin_fmaf(B.cqa, P[1] - P[5], B.cqd * (p26 + (P[8] - P[4])));
    const float pym = __builtin_fmaf(B.cqa, P[3] - P[7], B.cqd * (p26 + (P[4] - P[8])));
    qx_n = x.fpx + __builtin_fmaf(B.e, mxo, pxm);
    qy_n = x.fpy + __builtin_fmaf(B.e, myo, pym);
}

// Link product of node x with neighbour y: (h_x + h_y)(eta_y - eta_x).  The
// same link seen from y is exactly its negative, so each node computes its
// E, N, NE and NW links and takes the other four from its neighbours.
__device__ __forceinline__ float link(float hx, float ex, float hy, float ey)
{
    return (hx + hy) * (ey - ex);
}

// What one row of the window keeps: own values and the neighbours' values
// received across lanes.
struct Row {
    float eta, h, o3, o7;          // own
    float el, hl, o1l, o2l, o8l;   // from the lane on the left  (x - 1)
    float er, hr, o4r, o5r, o6r;   // from the lane on the right (x + 1)
};

__device__ __forceinline__ void exchange(const Derived& d, Row& R)
{
    R.eta = d.eta; R.h = d.h; R.o3 = d.o[3]; R.o7 = d.o[7];
    R.el = from_left(d.eta);   R.hl = from_left(d.h);
    R.o1l = from_left(d.o[1]); R.o2l = from_left(d.o[2]); R.o8l = from_left(d.o[8]);
    R.er = from_right(d.eta);  R.hr = from_right(d.h);
    R.o4r = from_right(d.o[4]); R.o5r = from_right(d.o[5]); R.o6r = from_right(d.o[6]);
}

struct Raw { float eta, qx, qy, H; };

// Index of a column / row to load: wrapped on periodic axes (lanes of a strip
// can reach up to 63 columns past the first one, more than n on narrow
// grids), clamped otherwise (values there only feed bounced links' lanes).
__device__ __forceinline__ int wrap_or_clamp(int r, int n, int periodic)
{
    if (periodic) {
        const int m = r % n;
        return m < 0 ? m + n : m;
    }
    return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

__device__ __forceinline__ bool is_open(int k) { return k == EDGE_DEPTH || k == EDGE_DISCHARGE; }

// ------------------------------------------------------------------ tile
// h = h_mean + amp - amp sin(omega t + phase), FP64
__device__ __forceinline__ double depth_bc(const BasinDev& B, int k, double tn)
{
    return B.bc_hmean[k] + B.bc_amp[k] - B.bc_amp[k] * sin(B.bc_om[k] * tn + B.bc_phase[k]);
}

// One output row r from window rows S (r-1), C (r), N (r+1).  WN holds the
// raw values of row r+1 and is refilled with row r+4.  Expanded three times
// in run_tile with rotated names (a macro rather than a function or lambda:
// every operand stays a plain local, so the whole window lives in registers).
#define MLB_ROW(r, WN, S, C, N, DC, DN)                                                           \
    do {                                                                                          \
        derive(B, WN.eta, WN.qx, WN.qy, WN.H, DN);                                                \
        exchange(DN, N);                                                                          \
        /* prefetch row r+4; rows past r1 are never needed (clamped: cache hits) */             \
        WN = load_raw(E0, QX0, QY0, HH,                                                           \
                      (uint32_t)(wrap_or_clamp(min((r) + 4, r1), ny, per_y) * ld) + (uint32_t)xl); \
        /* own links of row r (E, N, NE, NW) and the four received ones */                   \
        const float lE = link(DC.h, DC.eta, C.hr, C.er), lN = link(DC.h, DC.eta, N.h, N.eta);     \
        const float lNE = link(DC.h, DC.eta, N.hr, N.er), lNW = link(DC.h, DC.eta, N.hl, N.el);   \
        const float lWx = from_left(lE);                                                          \
        float P[9], oy[9];                                                                        \
        P[1] = -lWx; P[2] = -cNEl; P[3] = -cN; P[4] = -cNWr;                                      \
        P[5] = lE;   P[6] = lNE;   P[7] = lN;  P[8] = lNW;                                        \
        cN = lN; cNEl = from_left(lNE); cNWr = from_right(lNW); /* for row r+1 */                 \
        oy[1] = C.o1l; oy[2] = S.o2l; oy[3] = S.o3;  oy[4] = S.o4r;  /* W SW S SE */              \
        oy[5] = C.o5r; oy[6] = N.o6r; oy[7] = N.o7;  oy[8] = N.o8l;  /* E NE N NW */              \
        if (EDGE) {                                                                               \
            /* bounced link a: no bed term, A_a(y) = A_abar(x) */                                 \
            const bool sout = !per_y && (r) == 0, nout = !per_y && (r) == ny - 1;                 \
            const bool b2 = wout || sout, b4 = eout || sout, b6 = eout || nout, b8 = wout || nout; \
            P[1] = wout ? 0.0f : P[1]; oy[1] = wout ? DC.o[5] : oy[1];                            \
            P[2] = b2 ? 0.0f : P[2];   oy[2] = b2 ? DC.o[6] : oy[2];                              \
            P[3] = sout ? 0.0f : P[3]; oy[3] = sout ? DC.o[7] : oy[3];                            \
            P[4] = b4 ? 0.0f : P[4];   oy[4] = b4 ? DC.o[8] : oy[4];                              \
            P[5] = eout ? 0.0f : P[5]; oy[5] = eout ? DC.o[1] : oy[5];                            \
            P[6] = b6 ? 0.0f : P[6];   oy[6] = b6 ? DC.o[2] : oy[6];                              \
            P[7] = nout ? 0.0f : P[7]; oy[7] = nout ? DC.o[3] : oy[7];                            \
            P[8] = b8 ? 0.0f : P[8];   oy[8] = b8 ? DC.o[4] : oy[8];                              \
        }                                                                                         \
        float en, qxn, qyn;                                                                       \
        update(B, DC, P, oy, en, qxn, qyn);                                                       \
        bool store = own_col && (r) >= T.yo && (r) < r1;                                          \
        if (EDGE) {                                                                               \
            /* pre-override values of the x-neighbours (inward normals of W / E) */               \
            float re1 = 0.f, rx1 = 0.f, ry1 = 0.f, re2 = 0.f, rx2 = 0.f, ry2 = 0.f;               \
            float le1 = 0.f, lx1 = 0.f, ly1 = 0.f, le2 = 0.f, lx2 = 0.f, ly2 = 0.f;               \
            if (open_x) {                                                                         \
                re1 = from_right(en); rx1 = from_right(qxn); ry1 = from_right(qyn);               \
                re2 = from_right(re1); rx2 = from_right(rx1); ry2 = from_right(ry1);              \
                le1 = from_left(en); lx1 = from_left(qxn); ly1 = from_left(qyn);                  \
                le2 = from_left(le1); lx2 = from_left(lx1); ly2 = from_left(ly1);                 \
            }                                                                                     \
            const bool onS = !per_y && (r) == 0, onN = !per_y && (r) == ny - 1;                   \
            const bool wall = wall_x || (onS && kS == EDGE_WALL) || (onN && kN == EDGE_WALL);     \
            float fe = en, fx = qxn, fy = qyn;                                                    \
            if (wall) {                                                                           \
                fx = 0.0f; fy = 0.0f;                                                             \
            } else {                                                                              \
                /* a node lies on at most one open edge (adjacent open edges are rejected) */     \
                const bool oN = onN && is_open(kN);                                               \
                if (ox_lane || oN) {                                                              \
                    const float n1e = oW ? re1 : (oE ? le1 : h1e), n2e = oW ? re2 : (oE ? le2 : h2e); \
                    const float n1x = oW ? rx1 : (oE ? lx1 : h1x), n2x = oW ? rx2 : (oE ? lx2 : h2x); \
                    const float n1y = oW ? ry1 : (oE ? ly1 : h1y), n2y = oW ? ry2 : (oE ? ly2 : h2y); \
                    const float xe = two ? __builtin_fmaf(2.0f, n1e, -n2e) : n1e;                 \
                    const float xx = two ? __builtin_fmaf(2.0f, n1x, -n2x) : n1x;                 \
                    const float xy = two ? __builtin_fmaf(2.0f, n1y, -n2y) : n1y;                 \
                    const bool dep = oN ? kN == EDGE_DEPTH : dep_x;                               \
                    if (dep) {                                                                    \
                        fe = (float)((oN ? hbN : hb_x) - (double)DC.H); fx = xx; fy = xy;         \
                    } else {                                                                      \
                        fe = xe; fx = oN ? bqxN : bqx_x; fy = oN ? bqyN : bqy_x;                  \
                    }                                                                             \
                }                                                                                 \
            }                                                                                     \
            if (open_s) {                                                                         \
                if ((r) == 0) { /* row 0 waits for rows 1 (and 2) of this step */                 \
                    pe = en; pqx = qxn; pqy = qyn; pH = DC.H; poqx = DC.q0x; poqy = DC.q0y;       \
                    store = false;                                                                \
                } else if ((r) == extrap) {                                                       \
                    const float m1e = two ? h1e : en, m1x = two ? h1x : qxn, m1y = two ? h1y : qyn; \
                    const float ve = two ? __builtin_fmaf(2.0f, m1e, -en) : m1e;                  \
                    const float vx = two ? __builtin_fmaf(2.0f, m1x, -qxn) : m1x;                 \
                    const float vy = two ? __builtin_fmaf(2.0f, m1y, -qyn) : m1y;                 \
                    /* row-0 lanes are S-edge nodes or wall corners */                            \
                    float ge = pe, gx = pqx, gy = pqy;                                            \
                    if (wall_x) { gx = 0.0f; gy = 0.0f; }                                         \
                    else if (kS == EDGE_DEPTH) { ge = (float)(hbS - (double)pH); gx = vx; gy = vy; } \
                    else { ge = ve; gx = bqxS; gy = bqyS; }                                       \
                    if (own_col) {                                                                \
                        E1[x] = ge; QX1[x] = gx; QY1[x] = gy;                                     \
                        if (DIAG) account(sums, ge, gx, gy, pH, poqx, poqy);                      \
                    }                                                                             \
                }                                                                                 \
            }                                                                                     \
            h2e = h1e; h2x = h1x; h2y = h1y;                                                      \
            h1e = en;  h1x = qxn; h1y = qyn;                                                      \
            en = fe; qxn = fx; qyn = fy;                                                          \
        }                                                                                         \
        if (store) {                                                                              \
            const uint32_t o = ((uint32_t)((r) * ld) + (uint32_t)x) * 4u;                         \
            stf(E1, o, en); stf(QX1, o, qxn); stf(QY1, o, qyn);                                   \
            if (DIAG) account(sums, en, qxn, qyn, DC.H, DC.q0x, DC.q0y);                          \
        }                                                                                         \
    } while (0)

// Field access as SGPR base + 32-bit VGPR byte offset (one offset per row
// serves all fields).  Offsets fit in 32 bits: a plane holds < 2^30 floats.
typedef __attribute__((address_space(1))) const char gcbyte;
typedef __attribute__((address_space(1))) char gbyte;
__device__ __forceinline__ float ldf(const gfloat* base, uint32_t byte_off)
{
    return *(const gfloat*)((gcbyte*)base + byte_off);
}
__device__ __forceinline__ void stf(gfloat* base, uint32_t byte_off, float v)
{
#if MLB_NT_STORE
    __builtin_nontemporal_store(v, (gfloat*)((gbyte*)base + byte_off));
#else
    *(gfloat*)((gbyte*)base + byte_off) = v;
#endif
}

__device__ __forceinline__ Raw load_raw(const gfloat* __restrict__ E0, const gfloat* __restrict__ QX0,
                                        const gfloat* __restrict__ QY0, const gfloat* __restrict__ HH,
                                        uint32_t o)
{
    const uint32_t b = o * 4u;
    Raw w;
    w.eta = ldf(E0, b); w.qx = ldf(QX0, b); w.qy = ldf(QY0, b); w.H = ldf(HH, b);
    return w;
}

struct Sums { double eta, dq, q, bad, vmax; };

__device__ __forceinline__ void account(Sums& s, float en, float qxn, float qyn, float Hn, float oqx,
                                        float oqy)
{
    const double h = (double)Hn + (double)en;
    const bool ok = __builtin_isfinite(en) && __builtin_isfinite(qxn) && __builtin_isfinite(qyn) &&
                    h > 0.0;
    if (ok) {
        const double a = qxn, b = qyn, da = a - (double)oqx, db = b - (double)oqy;
        s.eta += en;
        s.dq += da * da + db * db;
        const double q2 = a * a + b * b;
        s.q += q2;
        const double sp = sqrt(q2) / h;
        s.vmax = sp > s.vmax ? sp : s.vmax;
    } else {
        s.bad += 1.0;
    }
}

// One wave's tile: the software-pipelined walk down the strip.
template <bool EDGE, bool DIAG>
__device__ __forceinline__ void run_tile(const BasinDev& B, const TileDev T, int rd,
                                         double* __restrict__ part)
{
    const int lane = threadIdx.x & (kWave - 1);
    const int nx = B.nx, ny = B.ny, ld = B.ld, per_y = B.per_y, extrap = B.extrap;
    const int x = T.x0 + lane - 1;
    const int xl = wrap_or_clamp(x, nx, B.per_x);
    const bool own_col = lane >= 1 && lane <= kStripOut && x >= T.xo && x < nx;
    const int wr = rd ^ 1;
    // fields are device (global) memory: typed so, loads and stores are
    // global_* instructions with exact wait counts rather than flat ones
    const gfloat* __restrict__ E0 = (const gfloat*)B.eta[rd];
    const gfloat* __restrict__ QX0 = (const gfloat*)B.qx[rd];
    const gfloat* __restrict__ QY0 = (const gfloat*)B.qy[rd];
    const gfloat* __restrict__ HH = (const gfloat*)B.H;
    gfloat* __restrict__ E1 = (gfloat*)B.eta[wr];
    gfloat* __restrict__ QX1 = (gfloat*)B.qx[wr];
    gfloat* __restrict__ QY1 = (gfloat*)B.qy[wr];

    // boundary data of this lane (edge tiles only)
    const int kW = B.kind[0], kE = B.kind[1], kS = B.kind[2], kN = B.kind[3];
    const bool two = extrap == 2;
    const bool wout = EDGE && !B.per_x && x == 0, eout = EDGE && !B.per_x && x == nx - 1;
    const bool wall_x = (wout && kW == EDGE_WALL) || (eout && kE == EDGE_WALL);
    const bool oW = wout && is_open(kW), oE = eout && is_open(kE), ox_lane = oW || oE;
    const bool dep_x = (oW && kW == EDGE_DEPTH) || (oE && kE == EDGE_DEPTH);
    double hbW = 0.0, hbE = 0.0, hbS = 0.0, hbN = 0.0;
    bool open_x = false, open_s = false;
    if (EDGE) {
        const double tn = (double)(B.stepc[rd] + 1) * B.dt;
        if (kW == EDGE_DEPTH) hbW = depth_bc(B, 0, tn);
        if (kE == EDGE_DEPTH) hbE = depth_bc(B, 1, tn);
        if (kS == EDGE_DEPTH) hbS = depth_bc(B, 2, tn);
        if (kN == EDGE_DEPTH) hbN = depth_bc(B, 3, tn);
        open_x = (is_open(kW) && T.x0 == 0) || (is_open(kE) && T.x0 + kStripOut >= nx);
        open_s = is_open(kS) && T.y0 == 0;
    }
    const double hb_x = oW ? hbW : hbE;
    const float bqx_x = oW ? B.bc_qx[0] : B.bc_qx[1], bqy_x = oW ? B.bc_qy[0] : B.bc_qy[1];
    const float bqxS = B.bc_qx[2], bqyS = B.bc_qy[2], bqxN = B.bc_qx[3], bqyN = B.bc_qy[3];
    // pre-override values of rows r-1, r-2 (open N edge) and the deferred row 0 (open S edge)
    float h1e = 0.f, h1x = 0.f, h1y = 0.f, h2e = 0.f, h2x = 0.f, h2y = 0.f;
    float pe = 0.f, pqx = 0.f, pqy = 0.f, pH = 0.f, poqx = 0.f, poqy = 0.f;
    Sums sums = {0.0, 0.0, 0.0, 0.0, 0.0};

    const int r0 = T.y0, r1 = T.y0 + T.rows;
    // Software pipeline: a row's raw values are loaded three rows before they
    // are derived.  Raw slots, window rows and derived nodes rotate with
    // period 3, so the loop is unrolled by 3 and the rotation is a renaming
    // (no register copy ever waits on a load in flight).
    Raw wa = load_raw(E0, QX0, QY0, HH, (uint32_t)(wrap_or_clamp(min(r0 + 1, r1), ny, per_y) * ld) + (uint32_t)xl);
    Raw wb = load_raw(E0, QX0, QY0, HH, (uint32_t)(wrap_or_clamp(min(r0 + 2, r1), ny, per_y) * ld) + (uint32_t)xl);
    Raw wc = load_raw(E0, QX0, QY0, HH, (uint32_t)(wrap_or_clamp(min(r0 + 3, r1), ny, per_y) * ld) + (uint32_t)xl);
    Derived d0, d1, d2;
    Row R0, R1, R2;
    {
        const Raw w = load_raw(E0, QX0, QY0, HH, (uint32_t)(wrap_or_clamp(min(r0 - 1, r1), ny, per_y) * ld) + (uint32_t)xl);
        derive(B, w.eta, w.qx, w.qy, w.H, d0);
        exchange(d0, R0);
    }
    {
        const Raw w = load_raw(E0, QX0, QY0, HH, (uint32_t)(wrap_or_clamp(min(r0, r1), ny, per_y) * ld) + (uint32_t)xl);
        derive(B, w.eta, w.qx, w.qy, w.H, d1);
        exchange(d1, R1);
    }
    // links of row r0-1 towards row r0, as row r0 receives them
    float cN = link(d0.h, d0.eta, R1.h, R1.eta);
    float cNEl = from_left(link(d0.h, d0.eta, R1.hr, R1.er));
    float cNWr = from_right(link(d0.h, d0.eta, R1.hl, R1.el));
    // single-exit counted loop: the tile's rows are rounded up to a multiple
    // of 3 and the pad rows (r >= r1) are computed but never stored
    const int nk = (T.rows + 2) / 3;
    int r = r0;
    for (int k = 0; k < nk; ++k, r += 3) {
        MLB_ROW(r, wa, R0, R1, R2, d1, d2);
        MLB_ROW(r + 1, wb, R1, R2, R0, d2, d0);
        MLB_ROW(r + 2, wc, R2, R0, R1, d0, d1);
    }
    if (DIAG) {
        // wave reduction in fixed order (xor butterfly), one partial set per tile
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) {
            sums.eta += __shfl_xor(sums.eta, off);
            sums.dq += __shfl_xor(sums.dq, off);
            sums.q += __shfl_xor(sums.q, off);
            sums.bad += __shfl_xor(sums.bad, off);
            const double vm = __shfl_xor(sums.vmax, off);
            sums.vmax = vm > sums.vmax ? vm : sums.vmax;
        }
        if (lane == 0) {
            part[0] = sums.eta; part[1] = sums.dq; part[2] = sums.q; part[3] = sums.bad;
            part[4] = sums.vmax; part[5] = 0.0;
        }
    }
}
#undef MLB_ROW

// ------------------------------------------------------------------ kernels
template <bool DIAG>
__global__ __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(DIAG ? 4 : 5)))
void step_kernel(const BasinDev* __restrict__ basins,
                                                      const TileDev* __restrict__ tiles, int ntiles,
                                                      int parity, double* __restrict__ partials)
{
    // One wave per tile, tiles in list order (largest basins first): the
    // hardware dispatcher hands out workgroups in index order, so the list is
    // consumed as a queue without a software loop.
    const int lane = threadIdx.x & (kWave - 1);
    const int t = uniform(blockIdx.x * (kBlock / kWave) + (threadIdx.x >> 6));
    if (t >= ntiles) return;
    const TileDev T = tiles[t];
    const BasinDev& B = basins[T.basin];
    const int rd = parity ^ B.swap;
    if (t == B.first_tile && lane == 0) {
        // the step counter advances once per launch; nobody else reads [rd ^ 1] now
        volatile int64_t* sc = B.stepc;
        sc[rd ^ 1] = sc[rd] + 1;
    }
    const bool edge = (!B.per_x && (T.x0 == 0 || T.x0 + kStripOut >= B.nx)) ||
                      (!B.per_y && (T.y0 == 0 || T.y0 + T.rows >= B.ny));
    double* part = partials + (size_t)t * kPartials;
    if (edge) run_tile<true, DIAG>(B, T, rd, part);
    else run_tile<false, DIAG>(B, T, rd, part);
}

// Reduction of the current state (no step): same partial layout as the step.
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
    double s_eta = 0.0, s_dq = 0.0, s_q = 0.0, s_bad = 0.0, s_vmax = 0.0;
    if (own_col) {
        for (int r = T.yo; r < T.y0 + T.rows; ++r) {
            const size_t o = (size_t)r * B.ld + x;
            const float en = B.eta[cur][o], a = B.qx[cur][o], b = B.qy[cur][o];
            const double h = (double)B.H[o] + (double)en;
            if (__builtin_isfinite(en) && __builtin_isfinite(a) && __builtin_isfinite(b) && h > 0.0) {
                const double da = (double)a - (double)B.qx[prev][o];
                const double db = (double)b - (double)B.qy[prev][o];
                s_eta += en;
                s_dq += da * da + db * db;
                const double q2 = (double)a * a + (double)b * b;
                s_q += q2;
                const double sp = sqrt(q2) / h;
                s_vmax = sp > s_vmax ? sp : s_vmax;
            } else {
                s_bad += 1.0;
            }
        }
    }
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        s_eta += __shfl_xor(s_eta, off);
        s_dq += __shfl_xor(s_dq, off);
        s_q += __shfl_xor(s_q, off);
        s_bad += __shfl_xor(s_bad, off);
        const double vm = __shfl_xor(s_vmax, off);
        s_vmax = vm > s_vmax ? vm : s_vmax;
    }
    if (lane == 0) {
        double* part = partials + (size_t)t * kPartials;
        part[0] = s_eta; part[1] = s_dq; part[2] = s_q; part[3] = s_bad; part[4] = s_vmax; part[5] = 0.0;
    }
}

// Per-basin sum of the tile partials in a fixed order: lane l sums tiles
// l, l+64, ... of the basin, then a fixed butterfly across the wave.
__global__ __launch_bounds__(kWave) void finalize_kernel(const BasinDev* __restrict__ basins,
                                                         const double* __restrict__ partials,
                                                         double* __restrict__ out)
{
    const BasinDev& B = basins[blockIdx.x];
    const int lane = threadIdx.x;
    double s[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int i = lane; i < B.ntiles; i += kWave) {
        const double* p = partials + (size_t)(B.first_tile + i) * kPartials;
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
    if (lane == 0) {
        double* o = out + (size_t)blockIdx.x * 8;
        o[0] = s[0]; o[1] = s[1]; o[2] = s[2]; o[3] = s[3]; o[4] = s[4];
        o[5] = (double)B.stepc[0]; o[6] = (double)B.stepc[1]; o[7] = 0.0;
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
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<true>, kBlock, 0);
    else
        (void)hipOccupancyMaxActiveBlocksPerMultiprocessor(&n, step_kernel<false>, kBlock, 0);
    return n > 0 ? n : 1;
}

hipError_t launch_step(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity,
                       double* d_partials, int diag, int tblock, unsigned dyn_lds, hipStream_t s)
{
    // dyn_lds: unused dynamic LDS that caps resident workgroups per CU
    if (tblock != 1) return hipErrorInvalidValue;
    const int per = kBlock / kWave;
    const dim3 grid((ntiles + per - 1) / per);
    if (diag)
        hipLaunchKernelGGL(step_kernel<true>, grid, dim3(kBlock), dyn_lds, s, d_basins, d_tiles,
                           ntiles, parity, d_partials);
    else
        hipLaunchKernelGGL(step_kernel<false>, grid, dim3(kBlock), dyn_lds, s, d_basins, d_tiles,
                           ntiles, parity, d_partials);
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
                           double* d_out, hipStream_t s)
{
    hipLaunchKernelGGL(finalize_kernel, dim3(nbasins), dim3(kWave), 0, s, d_basins, d_partials, d_out);
    return hipGetLastError();
}

}  // namespace mlb
