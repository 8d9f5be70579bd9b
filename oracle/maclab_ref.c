/*
 * Plain FP64 CPU oracle of the MacLABSWE streaming-only step
 * (Zhou, "Macroscopic Lattice Boltzmann Method for Shallow Water Equations",
 * arXiv 1902.02999).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * GPU path is checked against.  Only the test suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it; the product path never does.
 * It shares no code, header, table or constant with the GPU library.
 *
 * It evaluates the paper's update literally, in double precision:
 *   - local equilibrium f_a^eq(h, u)                 Eq. (feq-full)
 *   - per-direction incoming quantity, tau = 1       Eq. (Mac.lb.3)
 *   - depth  h  = sum_a of it                        Eq. (Mac.lb.6)
 *   - momentum hu_i = sum_a e_ai of it               Eq. (Mac.lb.7)
 *   - force F_j at the link midpoint                 Eq. (force-CS)
 *   - force = wind - bed friction + Coriolis         Eqs. (SWE-force), (wind_u-stress), (bed-stress)
 *   - e = 6 nu / dx, dt = dx / e                     Eq. (mlb-viscosity)
 *   - bounce-back f_a^eq = f_abar^eq at walls         Section 3, text after the stability note
 * with these readings of the points the paper leaves open:
 *   - h-bar on a link is the old-time average of the two end nodes (Eq. h-bar),
 *     or, with hbar_implicit, the definition given with Eq. (feq-full): the
 *     receiving node's new-time depth and the upstream node's old one.  The
 *     new depth then enters its own update linearly (through the bed term
 *     only), so the implicit equation is solved exactly per node.
 *   - F at the link midpoint is the old-time average of the two end nodes
 *   - bounced links carry f_abar^eq of the node itself, no bed or force term
 *   - after the update: WALL nodes get q = 0; DEPTH nodes get h = h_bc(t+dt)
 *     and q extrapolated inward; DISCHARGE nodes get q = q_bc and the free
 *     surface extrapolated inward (precedence WALL > DISCHARGE > DEPTH).
 *   - irregular geometry (staircase bounce-back, as the circular basin of
 *     Section 4 needs) comes from an optional per-node kind: a SOLID node lies
 *     outside the water and keeps its values; a link whose upstream node is
 *     SOLID is bounced like a link that leaves the grid; a WALL node is updated
 *     and then gets q = 0.  The kind overrides the edge logic at that node
 *     (SOLID, then WALL), and nodes that an open edge extrapolates from must
 *     be FLUID.
 * No reordering, blocking or fusion beyond that: every node recomputes the
 * equilibria of its upstream neighbours from h, u.
 */
#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* D2Q9 lattice (Section 3): direction 0 is the rest particle; odd directions
 * are the axis velocities with C = 1/3, lambda = 1; even directions are the
 * diagonals with C = 1/12, lambda = 1/4.  Numbered counter-clockwise from
 * east, which makes the paper's south-wall bounce-back pairs (2,6), (3,7),
 * (4,8) the directions pointing north. */
static const int    EX[9]  = {0, 1, 1, 0, -1, -1, -1, 0, 1};
static const int    EY[9]  = {0, 0, 1, 1, 1, 0, -1, -1, -1};
static const double CA[9]  = {0.0, 1.0 / 3.0, 1.0 / 12.0, 1.0 / 3.0, 1.0 / 12.0,
                              1.0 / 3.0, 1.0 / 12.0, 1.0 / 3.0, 1.0 / 12.0};
static const double LAM[9] = {0.0, 1.0, 0.25, 1.0, 0.25, 1.0, 0.25, 1.0, 0.25};
static const int    OPP[9] = {0, 5, 6, 7, 8, 1, 2, 3, 4};

enum { REF_WALL = 0, REF_PERIODIC = 1, REF_DEPTH = 2, REF_DISCHARGE = 3 };
enum { NODE_FLUID = 0, NODE_WALL = 1, NODE_SOLID = 2 };
enum { REF_W = 0, REF_E = 1, REF_S = 2, REF_N = 3 };

typedef struct {
    int32_t nx, ny;
    double  e, dt, g;
    double  tx, ty;       /* wind stress divided by water density  [m^2/s^2] */
    double  cb;           /* bed friction coefficient C_b = g / C_z^2         */
    double  omega;        /* Coriolis parameter                               */
    int32_t edge[4];      /* W, E, S, N edge kinds                            */
    int32_t extrap_order; /* 1: zero gradient, 2: linear                      */
    int32_t pad_;
    double  bc_h_mean[4], bc_amp[4], bc_period[4], bc_phase[4];
    double  bc_qx[4], bc_qy[4];
    const uint8_t* kind;  /* optional node kinds [ny][nx] (NODE_*), or NULL   */
    int32_t hbar_implicit; /* 0: Eq. (h-bar); 1: new-time depth at the node   */
    int32_t pad2_;
} mref_problem;

static int kind_at(const mref_problem* p, int i, int j)
{
    return p->kind ? p->kind[(size_t)j * p->nx + i] : NODE_FLUID;
}

/* ---------------------------------------------------------------- lattice */

void mref_lattice(int* ex, int* ey, double* ca, double* lam, int* opp)
{
    for (int a = 0; a < 9; ++a) {
        ex[a] = EX[a]; ey[a] = EY[a]; ca[a] = CA[a]; lam[a] = LAM[a]; opp[a] = OPP[a];
    }
}

/* Eq. (mlb-viscosity): particle speed from the eddy viscosity; dt = dx / e. */
void mref_params_from_nu(double dx, double nu, double* e, double* dt)
{
    *e  = 6.0 * nu / dx;
    *dt = dx / *e;
}

/* Eq. (wind_u-stress) divided by the water density. */
void mref_wind_stress(double rho_air, double c_w, double rho_w, double uwx, double uwy,
                      double* tx, double* ty)
{
    double speed = sqrt(uwx * uwx + uwy * uwy);
    *tx = rho_air * c_w * uwx * speed / rho_w;
    *ty = rho_air * c_w * uwy * speed / rho_w;
}

/* Eq. (bed-stress): C_b = g / C_z^2. */
double mref_bed_coeff(double g, double cz) { return cz > 0.0 ? g / (cz * cz) : 0.0; }

/* Eq. (feq-full): the local equilibrium of direction a at depth h, velocity (u, v). */
double mref_feq(int a, double g, double e, double h, double u, double v)
{
    double e2 = e * e, uu = u * u + v * v;
    if (a == 0) return h * (1.0 - 5.0 * g * h / (6.0 * e2) - 2.0 * uu / (3.0 * e2));
    double eu = e * EX[a] * u + e * EY[a] * v; /* e_ai u_i */
    return LAM[a] * h * (g * h / (6.0 * e2) + eu / (3.0 * e2) + eu * eu / (2.0 * e2 * e2)
                         - uu / (6.0 * e2));
}

/* Prescribed depth on a DEPTH edge: h_mean + amp - amp sin(2 pi t / T + phase).
 * (The tidal inflow of the paper's first test has this form.) */
double mref_depth_bc(const mref_problem* p, int edge, double t)
{
    double arg = p->bc_period[edge] > 0.0 ? 2.0 * M_PI * t / p->bc_period[edge] : 0.0;
    return p->bc_h_mean[edge] + p->bc_amp[edge] - p->bc_amp[edge] * sin(arg + p->bc_phase[edge]);
}

/* ------------------------------------------------------------- node terms */

/* Eq. (SWE-force) at a node: wind - bed friction (Eq. bed-stress) + Coriolis. */
static void node_force(const mref_problem* p, double h, double qx, double qy, double* fx, double* fy)
{
    double u = qx / h, v = qy / h, s = sqrt(u * u + v * v);
    *fx = p->tx - p->cb * u * s + p->omega * h * v;
    *fy = p->ty - p->cb * v * s - p->omega * h * u;
}

/* Upstream neighbour of (i, j) in direction a, i.e. x - e_a dt.  Returns 0 when
 * it lies outside a non-periodic edge or is a SOLID node (the link is then
 * bounced). */
static int upstream(const mref_problem* p, int i, int j, int a, int* yi, int* yj)
{
    int ii = i - EX[a], jj = j - EY[a];
    if (ii < 0 || ii >= p->nx) {
        if (p->edge[REF_W] != REF_PERIODIC) return 0;
        ii = (ii + p->nx) % p->nx;
    }
    if (jj < 0 || jj >= p->ny) {
        if (p->edge[REF_S] != REF_PERIODIC) return 0;
        jj = (jj + p->ny) % p->ny;
    }
    if (kind_at(p, ii, jj) == NODE_SOLID) return 0;
    *yi = ii; *yj = jj;
    return 1;
}

/* Eqs. (Mac.lb.3), (Mac.lb.6), (Mac.lb.7): the new h, hu, hv at node (i, j)
 * before any boundary override, with the link depth
 *   h-bar = (h(x) + h(y)) / 2           (Eq. h-bar; trial == NULL), or
 *   h-bar = (*trial + h(y)) / 2         (*trial: a new-time depth at x). */
static void update_with(const mref_problem* p, const double* zb, const double* h,
                        const double* qx, const double* qy, int i, int j, const double* trial,
                        double out[3])
{
    const int nx = p->nx;
    const double g = p->g, e = p->e, e2 = e * e, dt = p->dt;
    size_t x = (size_t)j * nx + i;
    double hx = h[x], ux = qx[x] / hx, vx = qy[x] / hx, fxx, fxy;
    node_force(p, hx, qx[x], qy[x], &fxx, &fxy);

    double hn = mref_feq(0, g, e, hx, ux, vx), qxn = 0.0, qyn = 0.0;
    for (int a = 1; a <= 8; ++a) {
        int yi, yj;
        double s;
        if (upstream(p, i, j, a, &yi, &yj)) {
            size_t y = (size_t)yj * nx + yi;
            double hy = h[y], uy = qx[y] / hy, vy = qy[y] / hy, fyx, fyy;
            node_force(p, hy, qx[y], qy[y], &fyx, &fyy);
            double hxb = trial ? *trial : hx;
            double hbar = 0.5 * (hxb + hy);                  /* Eq. (h-bar) / implicit  */
            double fbx = 0.5 * (fxx + fyx), fby = 0.5 * (fxy + fyy); /* Eq. (force-CS) */
            s = mref_feq(a, g, e, hy, uy, vy)
                - g / e2 * CA[a] * hbar * (zb[x] - zb[y])
                + dt / e2 * CA[a] * (e * EX[a] * fbx + e * EY[a] * fby);
        } else {
            s = mref_feq(OPP[a], g, e, hx, ux, vx);          /* bounce-back            */
        }
        hn  += s;
        qxn += e * EX[a] * s;
        qyn += e * EY[a] * s;
    }
    out[0] = hn; out[1] = qxn; out[2] = qyn;
}

/* The new state at (i, j) before any boundary override.  With the implicit
 * h-bar the node's new depth h' appears in its own update only through the
 * bed terms of its non-bounced links, each -(g/e^2) C_a (h'/2)(zb(x) - zb(y)):
 * h' = G0 - kap h' with G0 the update at h' = 0 and
 * kap = (g / (2 e^2)) sum_a C_a (zb(x) - zb(y)), so h' = G0 / (1 + kap); the
 * discharge is then the update evaluated at that h'. */
static void pre_update(const mref_problem* p, const double* zb, const double* h,
                       const double* qx, const double* qy, int i, int j, double out[3])
{
    if (!p->hbar_implicit) {
        update_with(p, zb, h, qx, qy, i, j, NULL, out);
        return;
    }
    const double zero = 0.0;
    double g0[3];
    update_with(p, zb, h, qx, qy, i, j, &zero, g0);
    const size_t x = (size_t)j * p->nx + i;
    double kap = 0.0;
    for (int a = 1; a <= 8; ++a) {
        int yi, yj;
        if (upstream(p, i, j, a, &yi, &yj))
            kap += p->g / (2.0 * p->e * p->e) * CA[a] * (zb[x] - zb[(size_t)yj * p->nx + yi]);
    }
    const double hnew = g0[0] / (1.0 + kap);
    update_with(p, zb, h, qx, qy, i, j, &hnew, out);
    out[0] = hnew;
}

/* Which override applies at (i, j): returns the kind and the edge whose
 * inward normal is used; -1 for an interior node. */
static int node_kind(const mref_problem* p, int i, int j, int* which)
{
    int on[4] = {i == 0, i == p->nx - 1, j == 0, j == p->ny - 1};
    static const int order[3] = {REF_WALL, REF_DISCHARGE, REF_DEPTH};
    for (int k = 0; k < 3; ++k)
        for (int ed = 0; ed < 4; ++ed)
            if (on[ed] && p->edge[ed] == order[k]) { *which = ed; return order[k]; }
    return -1;
}

static const int NRM_X[4] = {1, -1, 0, 0};
static const int NRM_Y[4] = {0, 0, 1, -1};

/* Final value at (i, j): the update, then the boundary override (step (e)). */
static void final_update(const mref_problem* p, const double* zb, const double* h,
                         const double* qx, const double* qy, double t_new, int i, int j,
                         double out[3])
{
    const int nk = kind_at(p, i, j);
    size_t x = (size_t)j * p->nx + i;
    if (nk == NODE_SOLID) { out[0] = h[x]; out[1] = qx[x]; out[2] = qy[x]; return; }
    int ed = 0, kind = node_kind(p, i, j, &ed);
    pre_update(p, zb, h, qx, qy, i, j, out);
    if (nk == NODE_WALL) { out[1] = 0.0; out[2] = 0.0; return; }
    if (kind < 0) return;
    if (kind == REF_WALL) { out[1] = 0.0; out[2] = 0.0; return; }
    int i1 = i + NRM_X[ed], j1 = j + NRM_Y[ed];
    int i2 = i + 2 * NRM_X[ed], j2 = j + 2 * NRM_Y[ed];
    double n1[3], n2[3] = {0, 0, 0};
    pre_update(p, zb, h, qx, qy, i1, j1, n1);
    if (p->extrap_order == 2) pre_update(p, zb, h, qx, qy, i2, j2, n2);
    size_t b = (size_t)j * p->nx + i, b1 = (size_t)j1 * p->nx + i1, b2 = (size_t)j2 * p->nx + i2;
    if (kind == REF_DEPTH) {
        out[0] = mref_depth_bc(p, ed, t_new);
        if (p->extrap_order == 2) {
            out[1] = 2.0 * n1[1] - n2[1];
            out[2] = 2.0 * n1[2] - n2[2];
        } else {
            out[1] = n1[1];
            out[2] = n1[2];
        }
    } else { /* DISCHARGE: prescribed q, free surface zeta = h + z_b extrapolated */
        double z1 = n1[0] + zb[b1];
        double zeta = p->extrap_order == 2 ? 2.0 * z1 - (n2[0] + zb[b2]) : z1;
        out[0] = zeta - zb[b];
        out[1] = p->bc_qx[ed];
        out[2] = p->bc_qy[ed];
    }
}

/* ------------------------------------------------------------------- API */

/* Problem checks: paired periodic edges; node kinds in range; FLUID on every
 * open edge and on the inner lines it extrapolates from. */
static int check_problem(const mref_problem* p)
{
    if (!p || p->nx < 3 || p->ny < 3) return -1;
    if ((p->edge[REF_W] == REF_PERIODIC) != (p->edge[REF_E] == REF_PERIODIC)) return -1;
    if ((p->edge[REF_S] == REF_PERIODIC) != (p->edge[REF_N] == REF_PERIODIC)) return -1;
    if (!p->kind) return 0;
    for (int j = 0; j < p->ny; ++j)
        for (int i = 0; i < p->nx; ++i) {
            int k = kind_at(p, i, j);
            if (k > NODE_SOLID) return -1;
            if (k == NODE_FLUID) continue;
            int dist[4] = {i, p->nx - 1 - i, j, p->ny - 1 - j};
            for (int ed = 0; ed < 4; ++ed)
                if ((p->edge[ed] == REF_DEPTH || p->edge[ed] == REF_DISCHARGE) && dist[ed] <= p->extrap_order)
                    return -1;
        }
    return 0;
}

/* One step n -> n+1 with t_old = n dt.  Outputs must not alias inputs. */
int mref_step(const mref_problem* p, const double* zb, const double* h, const double* qx,
              const double* qy, double t_old, double* h1, double* qx1, double* qy1, int nthreads)
{
    if (check_problem(p)) return -1;
    const int nx = p->nx, ny = p->ny;
    const double t_new = t_old + p->dt;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            double o[3];
            final_update(p, zb, h, qx, qy, t_new, i, j, o);
            size_t x = (size_t)j * nx + i;
            h1[x] = o[0]; qx1[x] = o[1]; qy1[x] = o[2];
        }
    (void)nthreads;
    return 0;
}

/* The value node (i, j) takes after one step from the given state. */
int mref_node(const mref_problem* p, const double* zb, const double* h, const double* qx,
              const double* qy, double t_old, int i, int j, double out[3])
{
    if (check_problem(p) || i < 0 || j < 0 || i >= p->nx || j >= p->ny) return -1;
    final_update(p, zb, h, qx, qy, t_old + p->dt, i, j, out);
    return 0;
}

/* The map whose fixed point the implicit h-bar defines: node (i, j)'s update
 * (before boundary overrides) when its new-time depth in h-bar is taken to be
 * `trial`.  For checking the exact solve only. */
int mref_node_trial(const mref_problem* p, const double* zb, const double* h, const double* qx,
                    const double* qy, int i, int j, double trial, double out[3])
{
    if (check_problem(p) || i < 0 || j < 0 || i >= p->nx || j >= p->ny) return -1;
    update_with(p, zb, h, qx, qy, i, j, &trial, out);
    return 0;
}

/* nsteps steps in place, starting at step index step0 (t = step0 dt).
 * work must hold 3 nx ny doubles. */
int mref_run(const mref_problem* p, const double* zb, double* h, double* qx, double* qy,
             int64_t step0, int64_t nsteps, double* work, int nthreads)
{
    size_t n = (size_t)p->nx * p->ny;
    double *h1 = work, *qx1 = work + n, *qy1 = work + 2 * n;
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = mref_step(p, zb, h, qx, qy, (double)(step0 + s) * p->dt, h1, qx1, qy1, nthreads);
        if (rc) return rc;
        memcpy(h, h1, n * sizeof(double));
        memcpy(qx, qx1, n * sizeof(double));
        memcpy(qy, qy1, n * sizeof(double));
    }
    return 0;
}

/* Diagnostics in a fixed serial order: out = {mass, residual, max speed,
 * non-finite-or-dry count}.  mass = sum h dx^2; residual = |q1 - q0| / |q1|
 * over both components (0 when the numerator is 0).  SOLID nodes (kind may be
 * NULL) are not part of the water and are skipped. */
void mref_diag(int32_t nx, int32_t ny, double dx, const double* h1, const double* qx1,
               const double* qy1, const double* qx0, const double* qy0, const uint8_t* kind,
               double out[4])
{
    double mass = 0.0, num = 0.0, den = 0.0, vmax = 0.0, bad = 0.0;
    size_t n = (size_t)nx * ny;
    for (size_t x = 0; x < n; ++x) {
        if (kind && kind[x] == NODE_SOLID) continue;
        double hh = h1[x], a = qx1[x], b = qy1[x];
        if (!isfinite(hh) || !isfinite(a) || !isfinite(b) || hh <= 0.0) { bad += 1.0; continue; }
        mass += hh * dx * dx;
        if (qx0 && qy0) {
            double da = a - qx0[x], db = b - qy0[x];
            num += da * da + db * db;
        }
        den += a * a + b * b;
        double sp = sqrt(a * a + b * b) / hh;
        if (sp > vmax) vmax = sp;
    }
    out[0] = mass;
    out[1] = num > 0.0 ? sqrt(num) / sqrt(den) : 0.0;
    out[2] = vmax;
    out[3] = bad;
}

int mref_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------- eLABSWE (tau != 1)
 * The lattice Boltzmann equation the method starts from (Eq. lb.1, in the
 * pull form of Eq. lb.Mac.1): nine stored distributions per node, relaxed
 * with the single time tau and streamed,
 *   f_a(x, t+dt) = f*_a(y) - (g/e^2) C_a h-bar (zb(x) - zb(y)) + (dt/e^2) C_a e_a . F-bar,
 *   f*_a(n) = f_a(n) - (f_a(n) - f_a^eq(n)) / tau,   y = x - e_a dt,
 * with the same readings as the streaming-only step: h-bar and F-bar are
 * old-time link averages (Eq. h-bar); a link whose upstream node lies past a
 * wall edge or is SOLID takes the node's own f*_abar and no bed or force term;
 * SOLID nodes keep their distributions; WALL nodes (edges of kind WALL or the
 * mask's WALL nodes) end the step at equilibrium with zero velocity,
 * f_a := f_a^eq(h', 0), h' = sum_a f_a (their discharge is zero, as in the
 * streaming-only step).  Open (DEPTH / DISCHARGE) edges are not part of this
 * baseline.  With tau = 1, f*_a = f_a^eq and the step is the streaming-only
 * one (Eq. Mac.lb.3); the viscosity is nu = e^2 dt (2 tau - 1) / 6 (Eq. viscosity).
 * Distributions are stored [9][ny][nx]. */

static void elab_macro(const mref_problem* p, const double* f, size_t x, size_t n, double* h, double* qx,
                       double* qy)
{
    double hh = 0.0, a = 0.0, b = 0.0;
    for (int k = 0; k < 9; ++k) {
        double v = f[(size_t)k * n + x];
        hh += v;
        a += p->e * EX[k] * v;
        b += p->e * EY[k] * v;
    }
    *h = hh; *qx = a; *qy = b;
}

/* Post-collision value f*_a at node x. */
static double elab_post(const mref_problem* p, double tau, const double* f, size_t x, size_t n, int a)
{
    double h, qx, qy;
    elab_macro(p, f, x, n, &h, &qx, &qy);
    double fa = f[(size_t)a * n + x];
    return fa - (fa - mref_feq(a, p->g, p->e, h, qx / h, qy / h)) / tau;
}

static int elab_check(const mref_problem* p, double tau)
{
    if (check_problem(p) || !(tau > 0.5)) return -1;
    for (int k = 0; k < 4; ++k)
        if (p->edge[k] == REF_DEPTH || p->edge[k] == REF_DISCHARGE) return -1;
    return 0;
}

/* f := f^eq(h, q) at every node (the usual start from a macroscopic state). */
int mref_elab_init(const mref_problem* p, const double* h, const double* qx, const double* qy, double* f)
{
    if (check_problem(p)) return -1;
    size_t n = (size_t)p->nx * p->ny;
    for (size_t x = 0; x < n; ++x)
        for (int a = 0; a < 9; ++a) f[(size_t)a * n + x] = mref_feq(a, p->g, p->e, h[x], qx[x] / h[x], qy[x] / h[x]);
    return 0;
}

/* h, hu, hv of stored distributions (Eqs. fea-0-h, fea-0-v). */
int mref_elab_macro(const mref_problem* p, const double* f, double* h, double* qx, double* qy)
{
    if (check_problem(p)) return -1;
    size_t n = (size_t)p->nx * p->ny;
    for (size_t x = 0; x < n; ++x) elab_macro(p, f, x, n, &h[x], &qx[x], &qy[x]);
    return 0;
}

/* One eLABSWE step f -> f1 (no aliasing). */
int mref_elab_step(const mref_problem* p, double tau, const double* zb, const double* f, double* f1,
                   int nthreads)
{
    if (elab_check(p, tau)) return -1;
    const int nx = p->nx, ny = p->ny;
    const size_t n = (size_t)nx * ny;
    const double g = p->g, e = p->e, e2 = e * e, dt = p->dt;
#ifdef _OPENMP
    if (nthreads < 1) nthreads = 1;
#pragma omp parallel for schedule(static) num_threads(nthreads)
#endif
    for (int j = 0; j < ny; ++j)
        for (int i = 0; i < nx; ++i) {
            const size_t x = (size_t)j * nx + i;
            const int nk = kind_at(p, i, j);
            if (nk == NODE_SOLID) {
                for (int a = 0; a < 9; ++a) f1[(size_t)a * n + x] = f[(size_t)a * n + x];
                continue;
            }
            double hx, qxx, qyx, fxx, fxy;
            elab_macro(p, f, x, n, &hx, &qxx, &qyx);
            node_force(p, hx, qxx, qyx, &fxx, &fxy);
            double out[9];
            out[0] = elab_post(p, tau, f, x, n, 0);
            for (int a = 1; a <= 8; ++a) {
                int yi, yj;
                if (upstream(p, i, j, a, &yi, &yj)) {
                    const size_t y = (size_t)yj * nx + yi;
                    double hy, qxy, qyy, fyx, fyy;
                    elab_macro(p, f, y, n, &hy, &qxy, &qyy);
                    node_force(p, hy, qxy, qyy, &fyx, &fyy);
                    double hbar = 0.5 * (hx + hy);                          /* Eq. (h-bar)    */
                    double fbx = 0.5 * (fxx + fyx), fby = 0.5 * (fxy + fyy); /* Eq. (force-CS) */
                    out[a] = elab_post(p, tau, f, y, n, a)
                             - g / e2 * CA[a] * hbar * (zb[x] - zb[y])
                             + dt / e2 * CA[a] * (e * EX[a] * fbx + e * EY[a] * fby);
                } else {
                    out[a] = elab_post(p, tau, f, x, n, OPP[a]);            /* bounce-back    */
                }
            }
            int ed = 0;
            if (nk == NODE_WALL || node_kind(p, i, j, &ed) == REF_WALL) {
                double hn = 0.0;
                for (int a = 0; a < 9; ++a) hn += out[a];
                for (int a = 0; a < 9; ++a) out[a] = mref_feq(a, g, e, hn, 0.0, 0.0);
            }
            for (int a = 0; a < 9; ++a) f1[(size_t)a * n + x] = out[a];
        }
    (void)nthreads;
    return 0;
}

/* nsteps eLABSWE steps in place; work holds 9 nx ny doubles. */
int mref_elab_run(const mref_problem* p, double tau, const double* zb, double* f, int64_t nsteps, double* work,
                  int nthreads)
{
    size_t n9 = (size_t)9 * p->nx * p->ny;
    for (int64_t s = 0; s < nsteps; ++s) {
        int rc = mref_elab_step(p, tau, zb, f, work, nthreads);
        if (rc) return rc;
        memcpy(f, work, n9 * sizeof(double));
    }
    return 0;
}
