// Device code of the MacLABSWE streaming-only step (Zhou, arXiv 1902.02999),
// shared by the one-step (mlb_kernels.hip) and two-step (mlb_kernels2.hip)
// kernel translation units.
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
//     - a bounced link (upstream outside a wall edge, or a SOLID node of the
//       optional geometry mask) takes A_abar(x) and no bed or force term,
//       i.e. the values of a virtual neighbour with eta_y = eta_x and
//       A_a(y) = A_abar(x); WALL nodes of the mask get q = 0 after the
//       update, SOLID nodes are never written.
//   With Out_a(n) = A_a built from q~(n), kk = 2K/(3e^2), K = q.u:
//     eta' = eta + sum_a Out_a(y_a) - kk + g/(2e^2) sum_a C_a P_a
//     q'   = (dt/2) F(x) + e sum_a e^_a Out_a(y_a) + g/(2e) sum_a C_a e^_a P_a
//   where P_a = (h_x + h_y)(eta_y - eta_x).
//   The sums are formed from partial sums in one fixed association order
//   (per neighbour row, see Row), so every code path gives the same bits.
//
// Execution: each wave walks a strip of columns down a tile of rows (a column
// per lane).  Per row it loads eta, qx, qy, H once (coalesced SoA rows),
// derives the node quantities once, and passes what its neighbours need
// across lanes with DPP wave shifts; a three-row register window gives the
// 8-neighbour gather.  One wave per tile; the tile list holds the largest
// basins first.
//   One step per pass: lanes 0 and 63 are the halo, 62 output columns.
//   Two steps per pass (temporal blocking): a first stage computes time level
//   n+1 for lanes 0..63 and hands each finished row, in registers, to a
//   second stage three rows behind it that computes level n+2; only lanes
//   2..61 (60 columns) are valid after two steps.  HBM traffic per step is
//   halved; level n+1 never leaves the registers.
//   Tiles whose window holds WALL or SOLID nodes of a mask take the edge path
//   with one extra byte per node (the kind) and a per-link bounce test; the
//   rest of a masked grid runs the ordinary paths.
#pragma once

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
__device__ __forceinline__ int from_left_i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x138 /* wave_shr:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ int from_right_i(int v)
{
    return __builtin_amdgcn_mov_dpp(v, 0x130 /* wave_shl:1 */, 0xf, 0xf, true);
}
__device__ __forceinline__ int uniform(int v) { return __builtin_amdgcn_readfirstlane(v); }

typedef __attribute__((address_space(1))) float gfloat;
typedef __attribute__((address_space(1))) double gdouble;

// ------------------------------------------------------------------ node arithmetic
struct Node {
    float eta, h, kq, fpx, fpy;       // kq = q . u
    float o[9];            // o[a] = Out_a(node), a = 1..8
    float H, q0x, q0y;     // the node's stored H and old discharge
    float iw, ikx, iky;    // implicit link depth: 1/(1+kappa), kappa_x, kappa_y
    float el;              // compensated surface: low part of eta
    int mk;                // masked tiles: node kind
};

// Node quantities from the old state (Eqs. SWE-force, bed-stress, feq-full).
// FRIC false: no bed friction (C_b = 0); the friction term is then exactly
// zero for finite states and is not evaluated.  COR false: no Coriolis force
// (Omega = 0); the term Omega q is then exactly zero and adding it changes no
// bit (the host stores the wind terms without a negative zero), so it is not
// evaluated either.
template <bool FRIC, bool COR = true>
__device__ __forceinline__ void derive(const BasinDev& B, float eta, float qx, float qy, float H, Node& d)
{
    const float h = H + eta;
    const float r = __builtin_amdgcn_rcpf(h);
    const float u = qx * r, v = qy * r;
    // (dt/2) F = (dt/2) [tau_w/rho - C_b u |u| + Omega (qy, -qx)]
    float fpx, fpy;
    if (FRIC) {
        const float s = __builtin_amdgcn_sqrtf(__builtin_fmaf(u, u, v * v));
        const float fr = B.cfr * s;
        fpx = __builtin_fmaf(-fr, u, B.tpx);
        fpy = __builtin_fmaf(-fr, v, B.tpy);
    } else {
        fpx = B.tpx;
        fpy = B.tpy;
    }
    if (COR) {
        fpx = __builtin_fmaf(B.omh, qy, fpx);
        fpy = __builtin_fmaf(-B.omh, qx, fpy);
    }
    // Out_a = quadratic part + linear part, each product fused into the sum
    // that uses it (every kernel variant evaluates this one expression)
    const float tqx = qx + fpx, tqy = qy + fpy;
    const float pxx = qx * u, pyy = qy * v, pxy = qx * v;
    const float kq = pxx + pyy;
    const float lx = B.c3e * tqx, ly = B.c3e * tqy;
    const float txx = __builtin_fmaf(2.0f, pxx, -pyy), tyy = __builtin_fmaf(2.0f, pyy, -pxx);
    const float rxy = B.c4 * pxy;
    const float qd1 = __builtin_fmaf(B.c12, kq, rxy), qd2 = __builtin_fmaf(B.c12, kq, -rxy);
    const float sp = lx + ly, sm = lx - ly;
    d.o[0] = 0.0f;
    d.o[1] = __builtin_fmaf(B.c6, txx, lx);     d.o[5] = __builtin_fmaf(B.c6, txx, -lx);
    d.o[3] = __builtin_fmaf(B.c6, tyy, ly);     d.o[7] = __builtin_fmaf(B.c6, tyy, -ly);
    d.o[2] = __builtin_fmaf(0.25f, sp, qd1);    d.o[6] = __builtin_fmaf(-0.25f, sp, qd1);
    d.o[4] = __builtin_fmaf(-0.25f, sm, qd2);   d.o[8] = __builtin_fmaf(0.25f, sm, qd2);
    d.eta = eta; d.h = h; d.kq = kq; d.fpx = fpx; d.fpy = fpy;
    d.H = H; d.q0x = qx; d.q0y = qy;
}

// Link product of node x with neighbour y: (h_x + h_y)(eta_y - eta_x).  The
// same link seen from y is exactly its negative, so each node computes its
// E, N, NE and NW links and takes the other four from its neighbours.
__device__ __forceinline__ float link(float hx, float ex, float hy, float ey)
{
    return (hx + hy) * (ey - ex);
}

// What one row of the window passes on: own depth and surface, the lane
// neighbours' (for the links), and the partial sums of the particles it sends
// to other rows, in the fixed order the update uses:
//   to the row above  S1 = (o2(x-1) + o3(x)) + o4(x+1),  S2 = o2(x-1) - o4(x+1)
//   to the row below  N1 = (o6(x+1) + o7(x)) + o8(x-1),  N2 = o8(x-1) - o6(x+1)
//   along the row     E1 = o1(x-1) + o5(x+1),            E2 = o1(x-1) - o5(x+1)
// Edge tiles keep the individual particles instead (bounced links replace
// some of them) and form the same sums at the receiving node.
// Lane shifts are written at each use (not stored), so the compiler folds
// each into the add or subtract that consumes it (a DPP source operand)
// instead of spending a separate move.
struct Row {
    float eta, h;
    float S1, S2, N1, N2, E1, E2;
    float o1l, o5r, o2l, o3, o4r, o6r, o7, o8l;
    int mk, ms;            // masked tiles: node kind; SOLID at x-1, x, x+1 (bits 0, 1, 2)
    float el;              // compensated surface: low part of eta
};

template <bool EDGE>
__device__ __forceinline__ void exchange(const Node& d, Row& R)
{
    R.eta = d.eta; R.h = d.h;
    if (EDGE) {
        R.o1l = from_left(d.o[1]); R.o5r = from_right(d.o[5]);
        R.o2l = from_left(d.o[2]); R.o3 = d.o[3]; R.o4r = from_right(d.o[4]);
        R.o6r = from_right(d.o[6]); R.o7 = d.o[7]; R.o8l = from_left(d.o[8]);
        R.S1 = R.S2 = R.N1 = R.N2 = R.E1 = R.E2 = 0.0f;
    } else {
        R.S1 = (from_left(d.o[2]) + d.o[3]) + from_right(d.o[4]);
        R.S2 = from_left(d.o[2]) - from_right(d.o[4]);
        R.N1 = (from_right(d.o[6]) + d.o[7]) + from_left(d.o[8]);
        R.N2 = from_left(d.o[8]) - from_right(d.o[6]);
        R.E1 = from_left(d.o[1]) + from_right(d.o[5]);
        R.E2 = from_left(d.o[1]) - from_right(d.o[5]);
        R.o1l = R.o5r = R.o2l = R.o3 = R.o4r = R.o6r = R.o7 = R.o8l = 0.0f;
    }
}

// Node kinds of a row in a masked tile: its own kind and which of the nodes
// x-1, x, x+1 are SOLID (their links into x are bounced).
__device__ __forceinline__ void mask_row(int m, Row& R)
{
    const int s = m == NODE_SOLID ? 1 : 0;
    R.mk = m;
    R.ms = from_left_i(s) | (s << 1) | (from_right_i(s) << 2);
}

// Link of node x with the lane neighbour of row R on its right / left.
__device__ __forceinline__ float link_right(float hx, float ex, const Row& R)
{
    return (hx + from_right(R.h)) * (from_right(R.eta) - ex);
}
__device__ __forceinline__ float link_left(float hx, float ex, const Row& R)
{
    return (hx + from_left(R.h)) * (from_left(R.eta) - ex);
}

// Compensated surface (eta = eta_hi + eta_lo, both FP32): the surface
// difference of a link is (ey - ex) + (ly - lx), the low parts restoring what
// rounding eta to FP32 loses.
__device__ __forceinline__ float link_c(float hx, float ex, float lx, float hy, float ey, float ly)
{
    return (hx + hy) * ((ey - ex) + (ly - lx));
}
__device__ __forceinline__ float link_right_c(float hx, float ex, float lx, const Row& R)
{
    return (hx + from_right(R.h)) * ((from_right(R.eta) - ex) + (from_right(R.el) - lx));
}
__device__ __forceinline__ float link_left_c(float hx, float ex, float lx, const Row& R)
{
    return (hx + from_left(R.h)) * ((from_left(R.eta) - ex) + (from_left(R.el) - lx));
}

// Links a row passes to the row above: its N link at x and its NE / NW links
// as the node above at x receives them (from x-1 and x+1).  Interior tiles
// keep their sum and difference, edge tiles the two values.
struct Carry { float cN, cBd, cBx, cNEl, cNWr; };

template <bool EDGE>
__device__ __forceinline__ void carry_from(float lN, float lNE, float lNW, Carry& c)
{
    const float a = from_left(lNE), b = from_right(lNW);
    c.cN = lN;
    if (EDGE) { c.cNEl = a; c.cNWr = b; c.cBd = 0.0f; c.cBx = 0.0f; }
    else { c.cBd = a + b; c.cBx = b - a; c.cNEl = 0.0f; c.cNWr = 0.0f; }
}

// Eqs. Mac.lb.6 / Mac.lb.7 in increment form, interior node.  With the link
// products P_1..P_8 (W SW S SE E NE N NW) of node x:
//   P1 = -lE(x-1), P2 = -lNE(x-1, row below), P3 = -lN(row below),
//   P4 = -lNW(x+1, row below), P5..P8 = lE, lNE, lN, lNW of x,
// the terms are the partial sums
//   Ha = P1 + P5, Hx = P1 - P5, Bd = P2 + P4, Bx = P2 - P4, Ud = P6 + P8, Ux = P8 - P6,
//   pa = (Ha + P3) + P7, pd = Bd + Ud,
//   mass: g/(6e^2) pa + g/(24e^2) pd,
//   x: g/(6e) Hx + g/(24e) (Bx + Ux),  y: g/(6e) (P3 - P7) + g/(24e) (Bd - Ud);
// each product is fused into the sum that takes it, in one fixed order:
//   eta increment = g/(6e^2) pa + (g/(24e^2) pd + (so - kk)),
//   qx = e mxo + (g/(6e) Hx + (g/(24e) (Bx + Ux) + (dt/2) Fx)), likewise qy.
// update_edge forms exactly these from the eight values, update_fast from
// the shared partial sums (equal bits: only exact negations differ).
//
// IMPL (implicit link depth, h-bar with the node's new depth): the new depth
// enters only through the bed terms, -(g/(2e^2)) C_a (h' - h) (z_x - z_y) more
// per link than with the old depth, so with the static per-node sums
// kappa = g/(2e^2) sum_a C_a (z_x - z_y) and kappa_v = g/(2e) sum_a C_a e^_a (z_x - z_y)
// over the non-bounced links the increment of the old-depth update is scaled
// by 1/(1+kappa) and the discharge loses increment * kappa_v.
//
// COMP (compensated surface): the increment joins the low part first and the
// new pair is renormalised exactly (Fast2Sum: |eta_hi| >= |inc + eta_lo|, or
// eta_hi = 0), so eta loses no more than FP32 rounding of the pair's sum.
template <bool IMPL, bool COMP>
__device__ __forceinline__ void finish(const Node& x, float inc, float& en, float& enl, float& qxn, float& qyn)
{
    if (IMPL) {
        inc = inc * x.iw;
        qxn = __builtin_fmaf(-inc, x.ikx, qxn);
        qyn = __builtin_fmaf(-inc, x.iky, qyn);
    }
    if (COMP) {
        const float s = inc + x.el;
        en = x.eta + s;
        enl = s - (en - x.eta);
    } else {
        en = x.eta + inc;
    }
}

template <bool IMPL, bool COMP>
__device__ __forceinline__ void update_fast(const BasinDev& B, const Node& x, const Row& S, const Row& C,
                                            const Row& N, const Carry& cy, float lE, float lN, float lNE,
                                            float lNW, float& en, float& enl, float& qxn, float& qyn)
{
    const float Ha = lE - from_left(lE), Hs = from_left(lE) + lE;   // Ha, -Hx
    const float Ud = lNE + lNW, Ux = lNW - lNE;
    const float pa = (Ha - cy.cN) + lN;
    const float pd = Ud - cy.cBd;                      // Bd = -cBd
    const float so = (C.E1 + S.S1) + N.N1;
    const float mxo = (C.E2 + S.S2) + N.N2;
    const float myo = S.S1 - N.N1;
    qxn = __builtin_fmaf(B.e, mxo, __builtin_fmaf(B.cqa, -Hs, __builtin_fmaf(B.cqd, cy.cBx + Ux, x.fpx)));
    qyn = __builtin_fmaf(B.e, myo, __builtin_fmaf(B.cqa, -(cy.cN + lN), __builtin_fmaf(B.cqd, -(cy.cBd + Ud), x.fpy)));
    finish<IMPL, COMP>(x, __builtin_fmaf(B.cma, pa, __builtin_fmaf(B.cmd, pd, __builtin_fmaf(-B.ckk, x.kq, so))),
                       en, enl, qxn, qyn);
}

// The same from the link products P[a] and gathered equilibria oy[a] = Out_a(y_a).
template <bool IMPL, bool COMP>
__device__ __forceinline__ void update_edge(const BasinDev& B, const Node& x, const float* P, const float* oy,
                                            float& en, float& enl, float& qxn, float& qyn)
{
    const float Ha = P[1] + P[5], Hx = P[1] - P[5];
    const float Bd = P[2] + P[4], Bx = P[2] - P[4];
    const float Ud = P[6] + P[8], Ux = P[8] - P[6];
    const float pa = (Ha + P[3]) + P[7];
    const float pd = Bd + Ud;
    const float E1 = oy[1] + oy[5], E2 = oy[1] - oy[5];
    const float S1 = (oy[2] + oy[3]) + oy[4], S2 = oy[2] - oy[4];
    const float N1 = (oy[6] + oy[7]) + oy[8], N2 = oy[8] - oy[6];
    const float so = (E1 + S1) + N1;
    const float mxo = (E2 + S2) + N2;
    const float myo = S1 - N1;
    qxn = __builtin_fmaf(B.e, mxo, __builtin_fmaf(B.cqa, Hx, __builtin_fmaf(B.cqd, Bx + Ux, x.fpx)));
    qyn = __builtin_fmaf(B.e, myo, __builtin_fmaf(B.cqa, P[3] - P[7], __builtin_fmaf(B.cqd, Bd - Ud, x.fpy)));
    finish<IMPL, COMP>(x, __builtin_fmaf(B.cma, pa, __builtin_fmaf(B.cmd, pd, __builtin_fmaf(-B.ckk, x.kq, so))),
                       en, enl, qxn, qyn);
}

struct Raw { float eta, qx, qy, H; int m; float iw, ikx, iky; float el; };   // m: node kind (masked tiles)

// Index of a column / row to load: wrapped on periodic axes (lanes of a strip
// can reach past the grid on narrow grids), clamped otherwise (values there
// only feed bounced links' lanes).
__device__ __forceinline__ int wrap_or_clamp(int r, int n, int periodic)
{
    if (periodic) {
        const int m = r % n;
        return m < 0 ? m + n : m;
    }
    return r < 0 ? 0 : (r >= n ? n - 1 : r);
}

__device__ __forceinline__ bool is_open(int k) { return k == EDGE_DEPTH || k == EDGE_DISCHARGE; }

// h = h_mean + amp - amp sin(omega t + phase), FP64
__device__ __forceinline__ double depth_bc(const BasinDev& B, int k, double tn)
{
    return B.bc_hmean[k] + B.bc_amp[k] - B.bc_amp[k] * sin(B.bc_om[k] * tn + B.bc_phase[k]);
}

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

typedef __attribute__((address_space(1))) const uint8_t gcu8;

// Static per-node planes of the implicit link depth.
struct Coef { const gfloat* w; const gfloat* kx; const gfloat* ky; };

template <bool MASK, bool IMPL, bool COMP>
__device__ __forceinline__ Raw load_raw(const gfloat* __restrict__ E0, const gfloat* __restrict__ QX0,
                                        const gfloat* __restrict__ QY0, const gfloat* __restrict__ HH,
                                        const gfloat* __restrict__ EL0, gcu8* __restrict__ MK, const Coef& K,
                                        uint32_t o)
{
    const uint32_t b = o * 4u;
    Raw w;
    w.eta = ldf(E0, b); w.qx = ldf(QX0, b); w.qy = ldf(QY0, b); w.H = ldf(HH, b);
    w.m = MASK ? (int)MK[o] : 0;
    if (IMPL) { w.iw = ldf(K.w, b); w.ikx = ldf(K.kx, b); w.iky = ldf(K.ky, b); }
    else { w.iw = 1.0f; w.ikx = 0.0f; w.iky = 0.0f; }
    w.el = COMP ? ldf(EL0, b) : 0.0f;
    return w;
}

template <bool IMPL, bool COMP>
__device__ __forceinline__ void take_coef(const Raw& w, Node& d)
{
    if (IMPL) { d.iw = w.iw; d.ikx = w.ikx; d.iky = w.iky; }
    d.el = COMP ? w.el : 0.0f;
}

// A lane's diagnostic sums over the nodes it stores: FP64 mass, residual
// numerator and denominator; the count of bad nodes and the largest speed in
// FP32 (a count per lane stays far below 2^24; the speed is a diagnostic).
struct Sums { double eta, dq, q; float bad, vmax; };

// COMP false: no low part of the surface (el is zero); the sum starts at +0
// and is never -0, so adding +0 would change no bit and is left out.
template <bool COMP = true>
__device__ __forceinline__ void account(Sums& s, float en, float qxn, float qyn, float Hn, float oqx,
                                        float oqy, float el)
{
    // the sign of the FP32 sum of two floats is exact, so Hn + en > 0 decides
    // h > 0 as the FP64 sum would
    const float hf = Hn + en;
    const bool ok = __builtin_isfinite(en) && __builtin_isfinite(qxn) && __builtin_isfinite(qyn) &&
                    hf > 0.0f;
    if (ok) {
        const double a = qxn, b = qyn, da = a - (double)oqx, db = b - (double)oqy;
        s.eta += en;
        if (COMP) s.eta += el;
        s.dq += da * da + db * db;
        s.q += a * a + b * b;
        const float sp = __builtin_amdgcn_sqrtf(qxn * qxn + qyn * qyn) * __builtin_amdgcn_rcpf(hf);
        s.vmax = sp > s.vmax ? sp : s.vmax;
    } else {
        s.bad += 1.0f;
    }
}

// Wave reduction of the lanes' sums in a fixed order (xor butterfly): one
// partial set per tile.
__device__ __forceinline__ void wave_partials(Sums& sums, double* __restrict__ part)
{
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
        sums.eta += __shfl_xor(sums.eta, off);
        sums.dq += __shfl_xor(sums.dq, off);
        sums.q += __shfl_xor(sums.q, off);
        sums.bad += __shfl_xor(sums.bad, off);
        const float vm = __shfl_xor(sums.vmax, off);
        sums.vmax = vm > sums.vmax ? vm : sums.vmax;
    }
    if ((threadIdx.x & (kWave - 1)) == 0) {
        part[0] = sums.eta; part[1] = sums.dq; part[2] = sums.q; part[3] = sums.bad;
        part[4] = sums.vmax; part[5] = 0.0;
    }
}

// Per-stage state of the walk: links carried to the next row, pre-override
// values of the two previous rows (open N edge), the deferred row 0 (open S
// edge) and the depth boundary values of the stage's time level.
struct Stage {
    Carry cy;
    float h1e, h1x, h1y, h2e, h2x, h2y;
    float pe, pqx, pqy, pH, poqx, poqy, pl;
    float piw, pikx, piky;   // implicit link depth: the deferred row's coefficients
    double hbS, hbN, hb_x;
};

// Lane and tile constants shared by the stages of one wave.
struct Lane {
    int x, xl;
    bool own_col, wout, eout, wall_x, oW, oE, ox_lane, dep_x, open_x, open_s, two;
    int kS, kN;
    float bqx_x, bqy_x, bqxS, bqyS, bqxN, bqyN;
};

// OPEN false: no lane of the tile reaches an open edge (walls and periodic
// edges only), so the open-edge logic is compiled out.
template <bool EDGE, bool OPEN>
__device__ __forceinline__ Lane lane_setup(const BasinDev& B, const TileDev& T, int x, bool own_lane, int xlo,
                                           int xhi)
{
    Lane L;
    const int nx = B.nx;
    L.x = x;
    L.xl = wrap_or_clamp(x, nx, B.per_x);
    L.own_col = own_lane && x >= T.xo && x < nx;
    const int kW = B.kind[0], kE = B.kind[1];
    L.kS = B.kind[2]; L.kN = B.kind[3];
    L.two = B.extrap == 2;
    L.wout = EDGE && !B.per_x && x == 0;
    L.eout = EDGE && !B.per_x && x == nx - 1;
    L.wall_x = (L.wout && kW == EDGE_WALL) || (L.eout && kE == EDGE_WALL);
    L.oW = OPEN && L.wout && is_open(kW);
    L.oE = OPEN && L.eout && is_open(kE);
    L.ox_lane = L.oW || L.oE;
    L.dep_x = (L.oW && kW == EDGE_DEPTH) || (L.oE && kE == EDGE_DEPTH);
    // some lane with valid values (columns xlo .. xhi) lies on an open W / E edge
    L.open_x = EDGE && OPEN && ((is_open(kW) && xlo <= 0) || (is_open(kE) && xhi >= nx - 1));
    L.open_s = EDGE && OPEN && is_open(L.kS) && T.y0 == 0;
    L.bqx_x = L.oW ? B.bc_qx[0] : B.bc_qx[1];
    L.bqy_x = L.oW ? B.bc_qy[0] : B.bc_qy[1];
    L.bqxS = B.bc_qx[2]; L.bqyS = B.bc_qy[2]; L.bqxN = B.bc_qx[3]; L.bqyN = B.bc_qy[3];
    return L;
}

template <bool EDGE, bool OPEN>
__device__ __forceinline__ void stage_setup(const BasinDev& B, const Lane& L, double tn, Stage& V)
{
    V.h1e = V.h1x = V.h1y = V.h2e = V.h2x = V.h2y = 0.0f;
    V.pe = V.pqx = V.pqy = V.pH = V.poqx = V.poqy = V.pl = 0.0f;
    V.piw = 1.0f; V.pikx = V.piky = 0.0f;
    V.hbS = V.hbN = V.hb_x = 0.0;
    if (EDGE && OPEN) {
        const int kW = B.kind[0], kE = B.kind[1];
        if (L.kS == EDGE_DEPTH) V.hbS = depth_bc(B, 2, tn);
        if (L.kN == EDGE_DEPTH) V.hbN = depth_bc(B, 3, tn);
        if (L.oW && kW == EDGE_DEPTH) V.hb_x = depth_bc(B, 0, tn);
        if (L.oE && kE == EDGE_DEPTH) V.hb_x = depth_bc(B, 1, tn);
    }
}

// Links of window row S towards row C (the first row of a walk).
template <bool EDGE, bool COMP>
__device__ __forceinline__ void carry_init(const Node& dS, const Row& C, Carry& cy)
{
    if (COMP)
        carry_from<EDGE>(link_c(dS.h, dS.eta, dS.el, C.h, C.eta, C.el), link_right_c(dS.h, dS.eta, dS.el, C),
                         link_left_c(dS.h, dS.eta, dS.el, C), cy);
    else
        carry_from<EDGE>(link(dS.h, dS.eta, C.h, C.eta), link_right(dS.h, dS.eta, C),
                         link_left(dS.h, dS.eta, C), cy);
}

// One output row r of a stage V from window rows S (r-1), C (r), N (r+1).
// RAWN holds the raw values of row r+1; LOADNEXT refills it (or nothing).
// EMIT(en, qxn, qyn, DC, enl) receives the row's new values and its old node
// (lanes decide ownership; enl is the new low part of a compensated surface);
// EMIT0(ge, gx, gy, gl) the deferred row 0 of an open S edge, once rows 1
// (and 2) exist.  A macro rather than a function or lambda: every operand stays a
// plain local, so the whole window lives in registers.
#define MLB_ROW(V, r, RAWN, S, C, N, DC, DN, LOADNEXT, EMIT, EMIT0)                                 \
    do {                                                                                          \
        derive<FRIC, COR>(B, RAWN.eta, RAWN.qx, RAWN.qy, RAWN.H, DN);                                   \
        take_coef<IMPL, COMP>(RAWN, DN);                                                          \
        exchange<EDGE>(DN, N);                                                                    \
        if (COMP) N.el = DN.el;                                                                   \
        if (MASK) { mask_row(RAWN.m, N); DN.mk = RAWN.m; }                                        \
        LOADNEXT;                                                                                 \
        const float lE = COMP ? link_right_c(DC.h, DC.eta, DC.el, C) : link_right(DC.h, DC.eta, C); \
        const float lN = COMP ? link_c(DC.h, DC.eta, DC.el, N.h, N.eta, N.el)                    \
                              : link(DC.h, DC.eta, N.h, N.eta);                                   \
        const float lNE = COMP ? link_right_c(DC.h, DC.eta, DC.el, N) : link_right(DC.h, DC.eta, N); \
        const float lNW = COMP ? link_left_c(DC.h, DC.eta, DC.el, N) : link_left(DC.h, DC.eta, N); \
        float en, enl = 0.0f, qxn, qyn;                                                           \
        if (EDGE) {                                                                               \
            float P[9], oy[9];                                                                    \
            P[1] = -from_left(lE); P[2] = -V.cy.cNEl; P[3] = -V.cy.cN; P[4] = -V.cy.cNWr;         \
            P[5] = lE;             P[6] = lNE;        P[7] = lN;       P[8] = lNW;                \
            oy[1] = C.o1l; oy[2] = S.o2l; oy[3] = S.o3;  oy[4] = S.o4r;  /* W SW S SE */          \
            oy[5] = C.o5r; oy[6] = N.o6r; oy[7] = N.o7;  oy[8] = N.o8l;  /* E NE N NW */          \
            /* bounced link a (upstream outside the grid or SOLID): no bed term,                  \
               A_a(y) = A_abar(x) */                                                              \
            const bool sout = !per_y && (r) == 0, nout = !per_y && (r) == ny - 1;                 \
            bool bb1_ = L.wout, bb2_ = L.wout || sout, bb3_ = sout, bb4_ = L.eout || sout;        \
            bool bb5_ = L.eout, bb6_ = L.eout || nout, bb7_ = nout, bb8_ = L.wout || nout;        \
            if (MASK) {                                                                           \
                bb1_ = bb1_ || (C.ms & 1); bb5_ = bb5_ || (C.ms & 4);                             \
                bb2_ = bb2_ || (S.ms & 1); bb3_ = bb3_ || (S.ms & 2); bb4_ = bb4_ || (S.ms & 4);  \
                bb8_ = bb8_ || (N.ms & 1); bb7_ = bb7_ || (N.ms & 2); bb6_ = bb6_ || (N.ms & 4);  \
            }                                                                                     \
            P[1] = bb1_ ? 0.0f : P[1];     oy[1] = bb1_ ? DC.o[5] : oy[1];                        \
            P[2] = bb2_ ? 0.0f : P[2];     oy[2] = bb2_ ? DC.o[6] : oy[2];                        \
            P[3] = bb3_ ? 0.0f : P[3];     oy[3] = bb3_ ? DC.o[7] : oy[3];                        \
            P[4] = bb4_ ? 0.0f : P[4];     oy[4] = bb4_ ? DC.o[8] : oy[4];                        \
            P[5] = bb5_ ? 0.0f : P[5];     oy[5] = bb5_ ? DC.o[1] : oy[5];                        \
            P[6] = bb6_ ? 0.0f : P[6];     oy[6] = bb6_ ? DC.o[2] : oy[6];                        \
            P[7] = bb7_ ? 0.0f : P[7];     oy[7] = bb7_ ? DC.o[3] : oy[7];                        \
            P[8] = bb8_ ? 0.0f : P[8];     oy[8] = bb8_ ? DC.o[4] : oy[8];                        \
            update_edge<IMPL, COMP>(B, DC, P, oy, en, enl, qxn, qyn);                             \
        } else {                                                                                  \
            update_fast<IMPL, COMP>(B, DC, S, C, N, V.cy, lE, lN, lNE, lNW, en, enl, qxn, qyn);   \
        }                                                                                         \
        carry_from<EDGE>(lN, lNE, lNW, V.cy); /* for row r+1 */                                   \
        /* keep the row's arithmetic ahead of the ownership branch of EMIT */                     \
        asm volatile("" ::"v"(en), "v"(qxn), "v"(qyn));                                           \
        if (COMP) asm volatile("" ::"v"(enl));                                                    \
        bool emit = true;                                                                         \
        if (EDGE) {                                                                               \
            /* pre-override values of the x-neighbours (inward normals of W / E) */               \
            float re1 = 0.f, rx1 = 0.f, ry1 = 0.f, re2 = 0.f, rx2 = 0.f, ry2 = 0.f;               \
            float le1 = 0.f, lx1 = 0.f, ly1 = 0.f, le2 = 0.f, lx2 = 0.f, ly2 = 0.f;               \
            if (OPEN && L.open_x) {                                                               \
                re1 = from_right(en); rx1 = from_right(qxn); ry1 = from_right(qyn);               \
                re2 = from_right(re1); rx2 = from_right(rx1); ry2 = from_right(ry1);              \
                le1 = from_left(en); lx1 = from_left(qxn); ly1 = from_left(qyn);                  \
                le2 = from_left(le1); lx2 = from_left(lx1); ly2 = from_left(ly1);                 \
            }                                                                                     \
            const bool onS = !per_y && (r) == 0, onN = !per_y && (r) == ny - 1;                   \
            const bool wall = L.wall_x || (onS && L.kS == EDGE_WALL) || (onN && L.kN == EDGE_WALL) || \
                              (MASK && C.mk == NODE_WALL);                                        \
            float fe = en, fx = qxn, fy = qyn, fl = enl;                                          \
            if (wall) {                                                                           \
                fx = 0.0f; fy = 0.0f;                                                             \
            } else {                                                                              \
                /* a node lies on at most one open edge (adjacent open edges are rejected) */     \
                const bool oN = OPEN && onN && is_open(L.kN);                                     \
                if ((OPEN && L.ox_lane) || oN) {                                                  \
                    const float n1e = L.oW ? re1 : (L.oE ? le1 : V.h1e);                          \
                    const float n2e = L.oW ? re2 : (L.oE ? le2 : V.h2e);                          \
                    const float n1x = L.oW ? rx1 : (L.oE ? lx1 : V.h1x);                          \
                    const float n2x = L.oW ? rx2 : (L.oE ? lx2 : V.h2x);                          \
                    const float n1y = L.oW ? ry1 : (L.oE ? ly1 : V.h1y);                          \
                    const float n2y = L.oW ? ry2 : (L.oE ? ly2 : V.h2y);                          \
                    const float xe = L.two ? __builtin_fmaf(2.0f, n1e, -n2e) : n1e;               \
                    const float xx = L.two ? __builtin_fmaf(2.0f, n1x, -n2x) : n1x;               \
                    const float xy = L.two ? __builtin_fmaf(2.0f, n1y, -n2y) : n1y;               \
                    const bool dep = oN ? L.kN == EDGE_DEPTH : L.dep_x;                           \
                    if (dep) {                                                                    \
                        const double dv = (oN ? V.hbN : V.hb_x) - (double)DC.H;                   \
                        fe = (float)dv; fx = xx; fy = xy;                                         \
                        if (COMP) fl = (float)(dv - (double)fe);                                  \
                    } else {                                                                      \
                        /* the extrapolated surface is taken in FP32 */                           \
                        fe = xe; fx = oN ? L.bqxN : L.bqx_x; fy = oN ? L.bqyN : L.bqy_x; fl = 0.0f; \
                    }                                                                             \
                }                                                                                 \
            }                                                                                     \
            if (OPEN && L.open_s) {                                                               \
                if ((r) == 0) { /* row 0 waits for rows 1 (and 2) of this step */                 \
                    V.pe = en; V.pqx = qxn; V.pqy = qyn; V.pH = DC.H; V.poqx = DC.q0x; V.poqy = DC.q0y; \
                    V.pl = enl;                                                                   \
                    if (IMPL) { V.piw = DC.iw; V.pikx = DC.ikx; V.piky = DC.iky; }                \
                    emit = false;                                                                 \
                } else if ((r) == extrap) {                                                       \
                    const float m1e = L.two ? V.h1e : en, m1x = L.two ? V.h1x : qxn;              \
                    const float m1y = L.two ? V.h1y : qyn;                                        \
                    const float ve = L.two ? __builtin_fmaf(2.0f, m1e, -en) : m1e;                \
                    const float vx = L.two ? __builtin_fmaf(2.0f, m1x, -qxn) : m1x;               \
                    const float vy = L.two ? __builtin_fmaf(2.0f, m1y, -qyn) : m1y;               \
                    /* row-0 lanes are S-edge nodes or wall corners */                            \
                    float ge = V.pe, gx = V.pqx, gy = V.pqy, gl = V.pl;                           \
                    if (L.wall_x) { gx = 0.0f; gy = 0.0f; }                                       \
                    else if (L.kS == EDGE_DEPTH) {                                                \
                        const double dv = V.hbS - (double)V.pH;                                   \
                        ge = (float)dv; gx = vx; gy = vy;                                         \
                        if (COMP) gl = (float)(dv - (double)ge);                                  \
                    }                                                                             \
                    else { ge = ve; gx = L.bqxS; gy = L.bqyS; gl = 0.0f; }                        \
                    EMIT0(ge, gx, gy, gl);                                                        \
                }                                                                                 \
            }                                                                                     \
            if (OPEN) { /* history of the open N edge's extrapolation */                          \
                V.h2e = V.h1e; V.h2x = V.h1x; V.h2y = V.h1y;                                      \
                V.h1e = en;    V.h1x = qxn;   V.h1y = qyn;                                        \
            }                                                                                     \
            en = fe; qxn = fx; qyn = fy; enl = fl;                                                \
        }                                                                                         \
        if (XO) {                                                                                 \
            /* interior arithmetic on a tile whose only edges are open W / E ones: the values of  \
               an open-edge node are replaced whole (as in the edge path), from its inner        \
               neighbours' new values and the boundary data */                                    \
            const float re1 = from_right(en), rx1 = from_right(qxn), ry1 = from_right(qyn);       \
            const float re2 = from_right(re1), rx2 = from_right(rx1), ry2 = from_right(ry1);      \
            const float le1 = from_left(en), lx1 = from_left(qxn), ly1 = from_left(qyn);          \
            const float le2 = from_left(le1), lx2 = from_left(lx1), ly2 = from_left(ly1);         \
            if (L.ox_lane) {                                                                      \
                const float n1e = L.oW ? re1 : le1, n2e = L.oW ? re2 : le2;                       \
                const float n1x = L.oW ? rx1 : lx1, n2x = L.oW ? rx2 : lx2;                       \
                const float n1y = L.oW ? ry1 : ly1, n2y = L.oW ? ry2 : ly2;                       \
                const float xe = L.two ? __builtin_fmaf(2.0f, n1e, -n2e) : n1e;                   \
                const float xx = L.two ? __builtin_fmaf(2.0f, n1x, -n2x) : n1x;                   \
                const float xy = L.two ? __builtin_fmaf(2.0f, n1y, -n2y) : n1y;                   \
                if (L.dep_x) {                                                                    \
                    en = (float)(V.hb_x - (double)DC.H); qxn = xx; qyn = xy;                      \
                } else {                                                                          \
                    en = xe; qxn = L.bqx_x; qyn = L.bqy_x;                                        \
                }                                                                                 \
            }                                                                                     \
        }                                                                                         \
        if (emit) { EMIT(en, qxn, qyn, DC, enl); }                                                \
    } while (0)

#define MLB_NOTHING(...) do { } while (0)

// ------------------------------------------------------------------ one step per pass
// MASK: the tile's window holds WALL or SOLID nodes (EDGE tiles only).
// IMPL: the basin uses the implicit link depth (coefficient planes).
// COMP: the surface is a compensated pair (eta plane plus a low-part plane).
template <bool EDGE, bool DIAG, bool FRIC, bool MASK, bool IMPL, bool COMP>
__device__ __forceinline__ void run_tile(const BasinDev& B, const TileDev T, int rd, int64_t step,
                                         double* __restrict__ part)
{
    static_assert(EDGE || !MASK, "the mask logic lives in the edge path");
    const int lane = threadIdx.x & (kWave - 1);
    const int ny = B.ny, ld = B.ld, per_y = B.per_y, extrap = B.extrap;
    constexpr bool OPEN = EDGE;   // one-step edge tiles keep the general boundary logic
    constexpr bool XO = false;
    constexpr bool COR = true;
    const Lane L = lane_setup<EDGE, OPEN>(B, T, T.x0 + lane - 1, lane >= 1 && lane <= kStripOut, T.x0, T.x0 + kStripOut - 1);
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
    gcu8* __restrict__ MK = (gcu8*)B.mask;
    const Coef K = {(const gfloat*)B.cw, (const gfloat*)B.ckx, (const gfloat*)B.cky};
    const gfloat* __restrict__ EL0 = (const gfloat*)B.etal[rd];
    gfloat* __restrict__ EL1 = (gfloat*)B.etal[wr];
    Stage V;
    stage_setup<EDGE, OPEN>(B, L, (double)(step + 1) * B.dt, V);
    Sums sums = {0.0, 0.0, 0.0, 0.0f, 0.0f};

    const int r0 = T.y0, r1 = T.y0 + T.rows;
#define MLB_LD(row) load_raw<MASK, IMPL, COMP>(E0, QX0, QY0, HH, EL0, MK, K, (uint32_t)(wrap_or_clamp(min((row), r1), ny, per_y) * ld) + (uint32_t)L.xl)
    // Software pipeline: a row's raw values are loaded three rows before they
    // are derived.  Raw slots, window rows and derived nodes rotate with
    // period 3, so the loop is unrolled by 3 and the rotation is a renaming
    // (no register copy ever waits on a load in flight).
    Raw wa = MLB_LD(r0 + 1), wb = MLB_LD(r0 + 2), wc = MLB_LD(r0 + 3);
    Node d0, d1, d2;
    Row R0, R1, R2;
    {
        const Raw w = MLB_LD(r0 - 1);
        derive<FRIC>(B, w.eta, w.qx, w.qy, w.H, d0);
        take_coef<IMPL, COMP>(w, d0);
        exchange<EDGE>(d0, R0);
        if (COMP) R0.el = d0.el;
        if (MASK) { mask_row(w.m, R0); d0.mk = w.m; }
    }
    {
        const Raw w = MLB_LD(r0);
        derive<FRIC>(B, w.eta, w.qx, w.qy, w.H, d1);
        take_coef<IMPL, COMP>(w, d1);
        exchange<EDGE>(d1, R1);
        if (COMP) R1.el = d1.el;
        if (MASK) { mask_row(w.m, R1); d1.mk = w.m; }
    }
    carry_init<EDGE, COMP>(d0, R1, V.cy);
    int r = r0;
// SOLID nodes are never stored: both buffers hold their values already
#define MLB_STORE1(en_, qx_, qy_, D_, el_)                                                        \
    do {                                                                                          \
        if (L.own_col && r >= T.yo && r < r1 && !(MASK && D_.mk == NODE_SOLID)) {                 \
            const uint32_t o = ((uint32_t)(r * ld) + (uint32_t)L.x) * 4u;                         \
            stf(E1, o, en_); stf(QX1, o, qx_); stf(QY1, o, qy_);                                  \
            if (COMP) stf(EL1, o, el_);                                                           \
            if (DIAG) account<COMP>(sums, en_, qx_, qy_, D_.H, D_.q0x, D_.q0y, COMP ? el_ : 0.0f);      \
        }                                                                                         \
    } while (0)
#define MLB_STORE0(ge_, gx_, gy_, gl_)                                                            \
    do {                                                                                          \
        if (L.own_col) {                                                                          \
            const uint32_t o = (uint32_t)L.x * 4u;                                                \
            stf(E1, o, ge_); stf(QX1, o, gx_); stf(QY1, o, gy_);                                  \
            if (COMP) stf(EL1, o, gl_);                                                           \
            if (DIAG) account<COMP>(sums, ge_, gx_, gy_, V.pH, V.poqx, V.poqy, COMP ? gl_ : 0.0f);      \
        }                                                                                         \
    } while (0)
    // single-exit counted loop: the tile's rows are rounded up to a multiple
    // of 3 and the pad rows (r >= r1) are computed but never stored
    const int nk = (T.rows + 2) / 3;
    for (int k = 0; k < nk; ++k) {
        MLB_ROW(V, r, wa, R0, R1, R2, d1, d2, wa = MLB_LD(r + 4), MLB_STORE1, MLB_STORE0);
        ++r;
        MLB_ROW(V, r, wb, R1, R2, R0, d2, d0, wb = MLB_LD(r + 4), MLB_STORE1, MLB_STORE0);
        ++r;
        MLB_ROW(V, r, wc, R2, R0, R1, d0, d1, wc = MLB_LD(r + 4), MLB_STORE1, MLB_STORE0);
        ++r;
    }
#undef MLB_STORE1
#undef MLB_STORE0
#undef MLB_LD
    if (DIAG) wave_partials(sums, part);
}

// ------------------------------------------------------------------ two steps per pass
// Stage A computes level n+1 for rows r0-1 .. (lanes 0..63, valid 1..62) and
// leaves each row in a queue slot; stage B, three rows behind, computes
// level n+2 for rows r0 .. r1-1 from the queue and stores lanes 2..61.
// Queue slot of A's row ra: (ra - r0 + 1) mod 3.  A's row 0 of an open S edge
// is final only after A's row `extrap`, so B starts once A has done row r0+2.
// MASK: the tile's window holds WALL or SOLID nodes (EDGE tiles only); the
// kinds travel with stage A's rows through the queue to stage B.
// OPEN: some lane of the tile reaches an open edge (see lane_setup).
// XO: the tile's only edges are open W / E ones (EDGE false): interior
// arithmetic, then the open-edge nodes' values replaced as the edge path does.
// IMPL: the basin uses the implicit link depth; each node's coefficients
// travel with stage A's rows through the queue to stage B.
// DIAG: the second stage also reduces its stored level n+2 against level n+1
// (the queue rows) into the tile's FP64 partials, as the one-step checked pass
// does against its old state.
template <bool EDGE, bool FRIC, bool MASK, bool OPEN, bool IMPL, bool XO = false, bool DIAG = false,
          bool COR = true>
__device__ __forceinline__ void run_tile2(const BasinDev& B, const TileDev T, int rd, int64_t step,
                                          double* __restrict__ part = nullptr)
{
    static_assert(EDGE || !MASK, "the mask logic lives in the edge path");
    const int lane = threadIdx.x & (kWave - 1);
    const int ny = B.ny, ld = B.ld, per_y = B.per_y, extrap = B.extrap;
    constexpr bool COMP = false;   // grids with a compensated surface run one step per pass
    gcu8* __restrict__ MK = (gcu8*)B.mask;
    const Coef K = {(const gfloat*)B.cw, (const gfloat*)B.ckx, (const gfloat*)B.cky};
    const Lane L = lane_setup<EDGE || XO, OPEN>(B, T, T.x0 + lane - 2, lane >= 2 && lane <= kStripOut2 + 1, T.x0 - 1,
                                    T.x0 + kStripOut2);
    const int wr = rd ^ 1;
    const gfloat* __restrict__ E0 = (const gfloat*)B.eta[rd];
    const gfloat* __restrict__ QX0 = (const gfloat*)B.qx[rd];
    const gfloat* __restrict__ QY0 = (const gfloat*)B.qy[rd];
    const gfloat* __restrict__ HH = (const gfloat*)B.H;
    gfloat* __restrict__ E1 = (gfloat*)B.eta[wr];
    gfloat* __restrict__ QX1 = (gfloat*)B.qx[wr];
    gfloat* __restrict__ QY1 = (gfloat*)B.qy[wr];
    const double tn0 = (double)step * B.dt;
    Sums sums = {0.0, 0.0, 0.0, 0.0f, 0.0f};
    Stage SA, SB;
    stage_setup<EDGE || XO, OPEN>(B, L, tn0 + B.dt, SA);
    stage_setup<EDGE || XO, OPEN>(B, L, tn0 + 2.0 * B.dt, SB);

    const int r0 = T.y0, r1 = T.y0 + T.rows;
    const int alast = r1 + 1;     // last level-n row stage A reads
#define MLB_LD(row) load_raw<MASK, IMPL, false>(E0, QX0, QY0, HH, nullptr, MK, K, (uint32_t)(wrap_or_clamp(min((row), alast), ny, per_y) * ld) + (uint32_t)L.xl)
    // stage A: prefetch of rows r0 .. r0+2, window rows r0-2 (S) and r0-1 (C)
    Raw wa = MLB_LD(r0), wb = MLB_LD(r0 + 1), wc = MLB_LD(r0 + 2);
    Node a0, a1, a2;
    Row A0, A1, A2;
    {
        const Raw w = MLB_LD(r0 - 2);
        derive<FRIC, COR>(B, w.eta, w.qx, w.qy, w.H, a0);
        take_coef<IMPL, false>(w, a0);
        exchange<EDGE>(a0, A0);
        if (MASK) { mask_row(w.m, A0); a0.mk = w.m; }
    }
    {
        const Raw w = MLB_LD(r0 - 1);
        derive<FRIC, COR>(B, w.eta, w.qx, w.qy, w.H, a1);
        take_coef<IMPL, false>(w, a1);
        exchange<EDGE>(a1, A1);
        if (MASK) { mask_row(w.m, A1); a1.mk = w.m; }
    }
    carry_init<EDGE, false>(a0, A1, SA.cy);
    Raw q0, q1, q2;               // level n+1 rows handed from A to B
    Node b0, b1, b2;
    Row B0, B1, B2;
    int ra = r0 - 1;
    // every lane's row goes into the queue, SOLID nodes included (their values
    // only meet bounced links, and stage B does not store them)
#define MLB_QC(q_, D_) do { if (IMPL) { q_.iw = D_.iw; q_.ikx = D_.ikx; q_.iky = D_.iky; } } while (0)
#define MLB_Q0(en_, qx_, qy_, D_, el_) do { q0.eta = en_; q0.qx = qx_; q0.qy = qy_; q0.H = D_.H; if (MASK) q0.m = D_.mk; MLB_QC(q0, D_); } while (0)
#define MLB_Q1(en_, qx_, qy_, D_, el_) do { q1.eta = en_; q1.qx = qx_; q1.qy = qy_; q1.H = D_.H; if (MASK) q1.m = D_.mk; MLB_QC(q1, D_); } while (0)
#define MLB_Q2(en_, qx_, qy_, D_, el_) do { q2.eta = en_; q2.qx = qx_; q2.qy = qy_; q2.H = D_.H; if (MASK) q2.m = D_.mk; MLB_QC(q2, D_); } while (0)
    // A's deferred row 0 (open S edge: r0 == 0, so its slot is q1; nodes next
    // to an open edge are FLUID)
#define MLB_A0(ge_, gx_, gy_, gl_) do { q1.eta = ge_; q1.qx = gx_; q1.qy = gy_; q1.H = SA.pH; if (MASK) q1.m = NODE_FLUID; \
                                         if (IMPL) { q1.iw = SA.piw; q1.ikx = SA.pikx; q1.iky = SA.piky; } } while (0)
    MLB_ROW(SA, ra, wa, A0, A1, A2, a1, a2, wa = MLB_LD(ra + 4), MLB_Q0, MLB_A0);   // row r0-1
    ++ra;
    // B's window row r0-1
    derive<FRIC, COR>(B, q0.eta, q0.qx, q0.qy, q0.H, b0);
    take_coef<IMPL, false>(q0, b0);
    exchange<EDGE>(b0, B0);
    if (MASK) { mask_row(q0.m, B0); b0.mk = q0.m; }
    MLB_ROW(SA, ra, wb, A1, A2, A0, a2, a0, wb = MLB_LD(ra + 4), MLB_Q1, MLB_A0);   // row r0
    ++ra;
    MLB_ROW(SA, ra, wc, A2, A0, A1, a0, a1, wc = MLB_LD(ra + 4), MLB_Q2, MLB_A0);   // row r0+1
    ++ra;
    MLB_ROW(SA, ra, wa, A0, A1, A2, a1, a2, wa = MLB_LD(ra + 4), MLB_Q0, MLB_A0);   // row r0+2
    ++ra;
    // B's window row r0 (final now) and its links towards row r0-1
    derive<FRIC, COR>(B, q1.eta, q1.qx, q1.qy, q1.H, b1);
    take_coef<IMPL, false>(q1, b1);
    exchange<EDGE>(b1, B1);
    if (MASK) { mask_row(q1.m, B1); b1.mk = q1.m; }
    carry_init<EDGE, false>(b0, B1, SB.cy);

    int rb = r0;
#define MLB_STORE2(en_, qx_, qy_, D_, el_)                                                         \
    do {                                                                                          \
        if (L.own_col && rb >= T.yo && rb < r1 && !(MASK && D_.mk == NODE_SOLID)) {               \
            const uint32_t o = ((uint32_t)(rb * ld) + (uint32_t)L.x) * 4u;                        \
            stf(E1, o, en_); stf(QX1, o, qx_); stf(QY1, o, qy_);                                  \
            if (DIAG) account<false>(sums, en_, qx_, qy_, D_.H, D_.q0x, D_.q0y, 0.0f);                   \
        }                                                                                         \
    } while (0)
#define MLB_STORE20(ge_, gx_, gy_, gl_)                                                           \
    do {                                                                                          \
        if (L.own_col) {                                                                          \
            const uint32_t o = (uint32_t)L.x * 4u;                                                \
            stf(E1, o, ge_); stf(QX1, o, gx_); stf(QY1, o, gy_);                                  \
            if (DIAG) account<false>(sums, ge_, gx_, gy_, SB.pH, SB.poqx, SB.poqy, 0.0f);                \
        }                                                                                         \
    } while (0)
    // B row rb consumes A's row rb+1; then A computes row rb+3.  Tiles pad
    // their rows to 3 nk + 2: nk rounds of three (B, A) pairs, then B's last
    // two rows alone, which need no further A row (A ends at r1 when the
    // tile's rows are 2 mod 3).  Tiles with open edges, whose boundary state
    // leaves no registers for that tail, pad to 3 nk and let A run two rows
    // past the tile.  Pad rows and A's surplus rows are computed but never
    // stored.
    constexpr bool TAIL = !(EDGE && OPEN);
    const int nk = TAIL ? T.rows / 3 : (T.rows + 2) / 3;   // T.rows >= 4, so nk >= 1
    // One round: three (B, A) pairs, after which every rotating slot is back
    // in place.  The loop runs two rounds per iteration, so a raw slot's
    // register can alternate between rounds: stage A's window still holds a
    // slot's old eta and H when the slot's next row is loaded.
#define MLB_ROUND()                                                                                \
    do {                                                                                          \
        MLB_ROW(SB, rb, q2, B0, B1, B2, b1, b2, MLB_NOTHING(), MLB_STORE2, MLB_STORE20);          \
        ++rb;                                                                                     \
        MLB_ROW(SA, ra, wb, A1, A2, A0, a2, a0, wb = MLB_LD(ra + 4), MLB_Q1, MLB_NOTHING);        \
        ++ra;                                                                                     \
        MLB_ROW(SB, rb, q0, B1, B2, B0, b2, b0, MLB_NOTHING(), MLB_STORE2, MLB_STORE20);          \
        ++rb;                                                                                     \
        MLB_ROW(SA, ra, wc, A2, A0, A1, a0, a1, wc = MLB_LD(ra + 4), MLB_Q2, MLB_NOTHING);        \
        ++ra;                                                                                     \
        MLB_ROW(SB, rb, q1, B2, B0, B1, b0, b1, MLB_NOTHING(), MLB_STORE2, MLB_STORE20);          \
        ++rb;                                                                                     \
        MLB_ROW(SA, ra, wa, A0, A1, A2, a1, a2, wa = MLB_LD(ra + 4), MLB_Q0, MLB_NOTHING);        \
        ++ra;                                                                                     \
    } while (0)
    // (interior tiles only: the boundary paths carry more state and would
    // spill with two rounds in flight)
    constexpr bool TWO = !EDGE && !XO;
    int k = 0;
    if (TWO) {
        for (; k + 1 < nk; k += 2) {
            MLB_ROUND();
            MLB_ROUND();
        }
    }
    for (; k < nk; ++k) MLB_ROUND();
#undef MLB_ROUND
    if (TAIL) {
        MLB_ROW(SB, rb, q2, B0, B1, B2, b1, b2, MLB_NOTHING(), MLB_STORE2, MLB_STORE20);
        ++rb;
        MLB_ROW(SB, rb, q0, B1, B2, B0, b2, b0, MLB_NOTHING(), MLB_STORE2, MLB_STORE20);
    }
#undef MLB_STORE2
#undef MLB_STORE20
    if (DIAG) wave_partials(sums, part);
#undef MLB_Q0
#undef MLB_Q1
#undef MLB_Q2
#undef MLB_QC
#undef MLB_A0
#undef MLB_LD
}
#undef MLB_ROW

// ------------------------------------------------------------------ kernels
// One wave's share of a pass: tile t advances its basin by one step (KIND 1,
// with the fused reduction when DIAG) or two (KIND 2).  `step` reads the
// basin's step counter at buffer rd; the basin's first tile advances it.
// MASKED: the tile list may hold TILE_MASKED tiles (a separate kernel, so
// that grids without a mask keep the smaller register budget).  CLOSED: no
// basin of the launch has an open edge (two-step passes compile the
// open-edge logic out).
template <int KIND, bool DIAG, bool MASKED, bool IMPL, bool COMP, bool CLOSED, class StepRead>
__device__ __forceinline__ void pass_tile(const BasinDev* __restrict__ basins, const TileDev* __restrict__ tiles,
                                          int t, int parity, double* __restrict__ partials, StepRead step_at)
{
    const int lane = threadIdx.x & (kWave - 1);
    const TileDev T = tiles[t];
    const BasinDev& B = basins[T.basin];
    const int rd = parity ^ B.swap;
    const int64_t step = step_at(B, rd);
    if (t == (KIND == 2 ? B.first_tile2 : B.first_tile) && lane == 0) {
        // the counter advances once per pass; nobody else reads [rd ^ 1] now
        volatile int64_t* sc = B.stepc;
        sc[rd ^ 1] = step + KIND;
    }
    if (KIND == 1) {
        const bool edge = (!B.per_x && (T.x0 == 0 || T.x0 + kStripOut >= B.nx)) ||
                          (!B.per_y && (T.y0 == 0 || T.y0 + T.rows >= B.ny));
        double* part = partials + (size_t)t * kPartials;
        const bool masked = MASKED && (T.flags & TILE_MASKED) != 0;
        if (B.cfr != 0.0f) {
            if (masked) run_tile<true, DIAG, true, MASKED, IMPL, COMP>(B, T, rd, step, part);
            else if (edge) run_tile<true, DIAG, true, false, IMPL, COMP>(B, T, rd, step, part);
            else run_tile<false, DIAG, true, false, IMPL, COMP>(B, T, rd, step, part);
        } else {
            if (masked) run_tile<true, DIAG, false, MASKED, IMPL, COMP>(B, T, rd, step, part);
            else if (edge) run_tile<true, DIAG, false, false, IMPL, COMP>(B, T, rd, step, part);
            else run_tile<false, DIAG, false, false, IMPL, COMP>(B, T, rd, step, part);
        }
    } else {
        // a two-step tile needs the boundary logic when stage A's rows
        // r0-1 .. r1 or lanes 1..62 touch an edge; the open-edge part of it
        // only when some basin of the launch has an open edge
        const bool tw = !B.per_x && T.x0 < 2, te = !B.per_x && T.x0 + kStripOut2 + 2 > B.nx;
        const bool ty = !B.per_y && (T.y0 < 2 || T.y0 + T.rows + 2 > B.ny);
        const bool edge = tw || te || ty;
        // only open W / E edges in reach: interior arithmetic plus the edge
        // nodes' replacement (a wall or an S / N edge needs the edge path)
        const bool xo = !CLOSED && edge && !ty && (!tw || is_open(B.kind[0])) && (!te || is_open(B.kind[1]));
        const bool masked = MASKED && (T.flags & TILE_MASKED) != 0;
        constexpr bool OPEN = !CLOSED;
        double* part = DIAG ? partials + (size_t)t * kPartials : nullptr;
        if (B.cfr != 0.0f) {
            if (masked) run_tile2<true, true, MASKED, OPEN, IMPL, false, DIAG>(B, T, rd, step, part);
            else if (xo) run_tile2<false, true, false, true, IMPL, true, DIAG>(B, T, rd, step, part);
            else if (edge) run_tile2<true, true, false, OPEN, IMPL, false, DIAG>(B, T, rd, step, part);
            else if (B.omh == 0.0f) run_tile2<false, true, false, false, IMPL, false, DIAG, false>(B, T, rd, step, part);
            else run_tile2<false, true, false, false, IMPL, false, DIAG>(B, T, rd, step, part);
        } else {
            if (masked) run_tile2<true, false, MASKED, OPEN, IMPL, false, DIAG>(B, T, rd, step, part);
            else if (xo) run_tile2<false, false, false, true, IMPL, true, DIAG>(B, T, rd, step, part);
            else if (edge) run_tile2<true, false, false, OPEN, IMPL, false, DIAG>(B, T, rd, step, part);
            else if (B.omh == 0.0f) run_tile2<false, false, false, false, IMPL, false, DIAG, false>(B, T, rd, step, part);
            else run_tile2<false, false, false, false, IMPL, false, DIAG>(B, T, rd, step, part);
        }
    }
}

struct PlainStep {
    __device__ int64_t operator()(const BasinDev& B, int rd) const { return B.stepc[rd]; }
};

// A step number known when the pass starts (work-queue launches compute it
// from the basin's counter at the launch and the pass index).
struct FixedStep {
    int64_t s;
    __device__ int64_t operator()(const BasinDev&, int) const { return s; }
};

// The counter of the previous pass of a persistent launch was written by
// another workgroup: read it as an agent-scope atomic (a vector load).
struct CoherentStep {
    __device__ int64_t operator()(const BasinDev& B, int rd) const
    {
        return __hip_atomic_load(B.stepc + rd, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
};

}  // namespace mlb
