/*
 * mlb.h -- C ABI of the MI355X (gfx950) MacLABSWE library.
 *
 * MacLABSWE is the streaming-only ("tau = 1") lattice Boltzmann method for
 * the shallow water equations of J. G. Zhou, arXiv 1902.02999.  One step
 * rebuilds the depth h and the discharge (hu, hv) at every node from the
 * local equilibria of the rest node and its 8 upstream neighbours
 * (Eqs. Mac.lb.6 and Mac.lb.7), adds the centred bed-slope and force terms
 * (Eqs. Mac.lb.3, force-CS), applies bounce-back no-slip walls and imposes
 * macroscopic Dirichlet values directly (Section 3, simulation procedure
 * steps (a)-(e)).
 *
 * Conventions
 *   - Every call returns an mlb_status; nothing throws or aborts across the
 *     ABI.  mlb_last_error() gives a thread-local message for the last failure.
 *   - SI units.  Host fields are row-major [ny][ld] doubles with ld >= nx;
 *     node (i, j) sits at x = i dx, y = j dx; i runs west->east, j south->north.
 *   - Host arrays passed in are borrowed for the duration of the call and
 *     copied.  Handles belong to the caller until the matching *_destroy.
 *   - Device memory is owned by the library unless the caller supplies a
 *     workspace (mlb_grid_create); then the workspace must outlive the grid.
 *   - One HIP stream per context; calls on one grid are not thread-safe.
 *   - Fields live on the GPU in FP32 as the perturbation eta = h - H from the
 *     still-water depth H = zeta_ref - z_b, plus qx = hu, qy = hv.
 */
#ifndef MLB_H
#define MLB_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    MLB_OK = 0,
    MLB_E_INVAL = -1,          /* bad argument, size or handle               */
    MLB_E_NOMEM = -2,          /* device or host allocation failed           */
    MLB_E_DEVICE = -3,         /* a HIP call failed (message has the error)  */
    MLB_E_UNSTABLE = -4,       /* g * H_max > e^2: the step is unstable      */
    MLB_E_NONFINITE = -5,      /* a check found a non-finite value or h <= 0 */
    MLB_E_STATE = -6,          /* call not allowed in the object's state     */
    MLB_E_NOTCONVERGED = -7,   /* max_steps reached before the tolerance     */
    MLB_E_STALLED = -8         /* residual stopped falling (see mlb_set_stall_checks) */
} mlb_status;

/* Edge kinds.  Edges are indexed W=0 (i = 0), E=1 (i = nx-1), S=2 (j = 0),
 * N=3 (j = ny-1).  Boundary nodes are computational nodes of the lattice.
 *  WALL      no-slip wall: links from outside are bounced back
 *            (f_a^eq = f_abar^eq of the node itself), then hu = hv = 0
 *            (Section 3, the bounce-back example after the stability note).
 *  PERIODIC  the lattice wraps; must be set on both W and E, or on both S and N.
 *  DEPTH     h is imposed, h = h_mean + amp - amp sin(2 pi t / T + phase);
 *            the discharge is extrapolated from the inner nodes.
 *  DISCHARGE (hu, hv) is imposed; the free surface h + z_b is extrapolated
 *            from the inner nodes.
 * A node on two edges takes the kind WALL over DISCHARGE over DEPTH.  Two
 * adjacent edges may not both be open (DEPTH/DISCHARGE). */
enum { MLB_EDGE_WALL = 0, MLB_EDGE_PERIODIC = 1, MLB_EDGE_DEPTH = 2, MLB_EDGE_DISCHARGE = 3 };
enum { MLB_W = 0, MLB_E = 1, MLB_S = 2, MLB_N = 3 };

typedef struct {
    int32_t nx, ny;        /* nodes per direction, >= 4 each (>= 5 with open edges); nx
                              rounded up to a multiple of 64, times ny, < 2^30 (about
                              32768 x 32767 nodes, 4 GiB per field)                   */
    double  dx;            /* lattice size [m]                                             */
    double  nu;            /* eddy viscosity [m^2/s]; e = 6 nu / dx, dt = dx / e (Eq. mlb-viscosity) */
    double  g;             /* gravity, 9.81 in the paper                                   */
    double  rho_w;         /* water density for the stresses (not given in the paper)      */
    double  rho_air;       /* air density, 1.293 (Eq. wind_u-stress)                       */
    double  c_w;           /* wind drag coefficient, 0.0026 (Eq. wind_u-stress)            */
    double  omega;         /* Coriolis parameter (Eq. SWE-force)                           */
    double  zeta_ref;      /* still-water level: H = zeta_ref - z_b                        */
    int32_t edge[4];       /* W, E, S, N edge kinds                                        */
    int32_t extrap_order;  /* 1: zero-gradient, 2: linear extrapolation at open edges      */
} mlb_params;

/* Diagnostics of the last completed step (FP64, fixed summation order). */
typedef struct {
    int64_t step;          /* steps taken                                                  */
    double  t;             /* step * dt [s]                                                */
    double  mass;          /* sum of h dx^2 over all nodes but SOLID ones [m^3]            */
    double  residual;      /* |q(n) - q(n-1)|_2 / |q(n)|_2, both components; 0 if no change */
    double  max_speed;     /* max |q| / h [m/s]                                            */
    int64_t nonfinite;     /* nodes with a non-finite value or h <= 0                      */
    double  e, dt;         /* lattice speed [m/s] and time step [s]                         */
    double  gh_over_e2;    /* g * H_max / e^2 (must stay <= 1)                             */
    double  rle;           /* lattice Reynolds number max_speed * dx / nu (< 1 advised)    */
} mlb_diag_t;

typedef struct mlb_ctx   mlb_ctx;
typedef struct mlb_grid  mlb_grid;
typedef struct mlb_batch mlb_batch;

/* Status text and the calling thread's last error message (never NULL). */
const char* mlb_status_str(mlb_status s);
const char* mlb_last_error(void);

/* A context binds one GPU and one HIP stream.  stream == NULL: the library
 * creates its own stream (default priority).  Otherwise the caller's
 * hipStream_t is used and must outlive the context. */
mlb_status mlb_ctx_create(int device, void* hip_stream, mlb_ctx** out);
/* MLB_E_STATE while grids or batches created from it are alive. */
mlb_status mlb_ctx_destroy(mlb_ctx* ctx);
/* Blocks until the context's stream is idle.  MLB_E_DEVICE if a persistent
 * launch on the context gave up at a pass barrier since the last check. */
mlb_status mlb_ctx_sync(mlb_ctx* ctx);
/* Stall rule of the steady-state runs on this context (mlb_run_steady,
 * mlb_warm_start_run): with checks > 0 a run stops with MLB_E_STALLED once
 * the smallest residual seen so far is within a factor 10 of the tolerance
 * and `checks` consecutive checks have not lowered it.  FP32 fields put a
 * noise floor under the residual that can sit at a tolerance like 1e-6; the
 * state is then as steady as FP32 holds it.  0 (default): off. */
mlb_status mlb_set_stall_checks(mlb_ctx* ctx, int32_t checks);

/* Device bytes of a grid's fields (two copies of eta, qx, qy; the still-water
 * depth; a 256-byte header with the step counter and the last step's
 * diagnostic sums) for a caller-owned workspace.  The small tile list
 * and reduction buffers are always allocated by the library. */
mlb_status mlb_grid_workspace_bytes(const mlb_params* p, size_t* bytes);
/* Creates a grid.  dev_workspace == NULL: the library allocates device memory.
 * Otherwise it must be a device pointer of at least mlb_grid_workspace_bytes,
 * 256-byte aligned, owned by the caller and kept alive until the grid is destroyed.
 * The new grid has a flat bed at zeta_ref - 1, still water and no forcing. */
mlb_status mlb_grid_create(mlb_ctx* ctx, const mlb_params* p, void* dev_workspace,
                           size_t ws_bytes, mlb_grid** out);
mlb_status mlb_grid_destroy(mlb_grid* g);

/* Bed elevation z_b [ny][ld] (host, copied).  Sets H = zeta_ref - z_b (FP64,
 * stored FP32), still water (eta = 0, q = 0) and resets the step counter.
 * MLB_E_UNSTABLE if g * max(H) > e^2 (linear stability of the step);
 * MLB_E_INVAL if some H <= 0 (no wetting/drying). */
mlb_status mlb_set_bathymetry(mlb_grid* g, const double* zb, int64_t ld);

/* Node kinds of the optional geometry mask: irregular basins by staircase
 * bounce-back (the bounce-back of Section 3 applied at every link that starts
 * at a SOLID node; the circular basin of Section 4 is built this way). */
enum { MLB_NODE_FLUID = 0, MLB_NODE_WALL = 1, MLB_NODE_SOLID = 2 };
/* Node kinds [ny][ld] (host, copied into a device byte plane that the library
 * allocates); kind == NULL removes the mask.
 *   FLUID  an ordinary node (the edge kinds apply as without a mask);
 *   WALL   updated, then q = 0 (no-slip boundary node);
 *   SOLID  outside the water: never written, left out of the diagnostics
 *          (mass, residual, max speed, non-finite count); a link whose
 *          upstream node is SOLID is bounced (f_a^eq := f_abar^eq of the node
 *          itself, no bed or force term), as at a wall edge.
 * A node's kind overrides its edge kind (SOLID, then WALL).  SOLID nodes
 * still need a positive H (its value is never used).  MLB_E_INVAL for a kind
 * above SOLID, for a non-FLUID node within extrap_order nodes of an open
 * (DEPTH / DISCHARGE) edge, or when every node is SOLID.  The current state
 * is copied into the second buffer set, so the next residual is 0.  Tiles
 * whose window holds WALL or SOLID nodes run a masked kernel variant (one or
 * two steps per pass); tiles owning only SOLID nodes are not launched.
 * MLB_E_STATE if the grid belongs to a live batch. */
mlb_status mlb_set_mask(mlb_grid* g, const uint8_t* kind, int64_t ld);

/* The wave tiles a grid of these parameters (and optional node kinds
 * [ny][kind_ld]) is stepped with, without a device: six int32 per tile,
 * (x0, y0, rows, xo, yo, flags).  A tile's wave covers columns x0 - k ..
 * x0 - k + 63 (k = 1 for one step per pass, 2 for two) and computes rows
 * y0 .. y0 + rows - 1; it stores the nodes of columns max(x0, xo) ..
 * x0 + 61 - (k - 1) * 2 (below nx) and rows yo .. y0 + rows - 1.  flags bit 0:
 * the tile's window holds a WALL or SOLID node (masked kernel path).  Tiles
 * that would own only SOLID nodes are left out.  The list is in dispatch
 * order: tiles on a non-periodic edge or with the masked flag first, then the
 * rest, each group band by band.  Writes at most `capacity` tiles; *count
 * receives the number of tiles.  No device memory is used. */
mlb_status mlb_plan_tiles(const mlb_params* p, const uint8_t* kind, int64_t kind_ld, int32_t tile_rows,
                          int32_t tblock, int32_t* tiles, int64_t capacity, int64_t* count);

/* The dependency lists the work-queue launches (mlb_exec_opts.persistent = 2)
 * of such a grid use, without a device, for the tile list of mlb_plan_tiles
 * (same arguments): the item of tile t in pass p waits until every tile
 * nbr[off[t]] .. nbr[off[t+1] - 1] (t itself included, ascending) has
 * completed pass p - 1.  They are the tiles owning a node of t's window (what
 * its wave loads) and the tiles whose window holds a node t owns.  Writes at
 * most off_capacity offsets (ntiles + 1 are needed) and nbr_capacity indices;
 * *ntiles and *nnbr receive the counts.  MLB_E_STATE if a tile would depend
 * on more than 64 tiles (such grids step with ordinary launches). */
mlb_status mlb_plan_workqueue(const mlb_params* p, const uint8_t* kind, int64_t kind_ld, int32_t tile_rows,
                              int32_t tblock, int32_t* off, int64_t off_capacity, int32_t* nbr,
                              int64_t nbr_capacity, int64_t* ntiles, int64_t* nnbr);

/* Link depth h-bar of the bed term (Section 3).
 *   SEMI_IMPLICIT  h-bar = (h(x,t) + h(x - e_a dt,t)) / 2, Eq. (h-bar): the
 *                  form the paper prefers; exact volume conservation and the
 *                  two-step kernel.  Default.
 *   IMPLICIT       h-bar = (h(x,t+dt) + h(x - e_a dt,t)) / 2, the definition
 *                  given with Eq. (feq-full): the receiving node's new depth.
 *                  It enters the node's update only through its bed terms, so
 *                  the equation is affine in it and is solved exactly per node
 *                  (static per-node sums over the non-bounced links,
 *                  recomputed by mlb_set_bathymetry and mlb_set_mask; 12 more
 *                  bytes per node read per step).  The volume is then
 *                  conserved only to O(dt) of the bed-term asymmetry.  Grids
 *                  in this form take one or two steps per pass (the
 *                  coefficients travel with the two-step kernel's rows) with
 *                  ordinary launches (persistent is accepted and runs as
 *                  graph / stream launches).
 * MLB_E_UNSTABLE if 1 + kappa <= 0 at some node (a bed far too rough for the
 * lattice); MLB_E_STATE if the grid belongs to a live batch.  The grids of a
 * batch must share the form (mlb_batch_create: MLB_E_INVAL otherwise). */
enum { MLB_HBAR_SEMI_IMPLICIT = 0, MLB_HBAR_IMPLICIT = 1 };
mlb_status mlb_set_hbar(mlb_grid* g, int32_t mode);

/* Storage precision of the surface perturbation eta = h - H.
 *   FP32         one FP32 plane per buffer (default; every kernel).
 *   COMPENSATED  eta is the unevaluated sum of two FP32 values (a second
 *                plane per buffer holds the low part): each update adds its
 *                increment to the low part and renormalises exactly, and link
 *                surface differences include the low parts.  For slow flows
 *                under a large surface range (a tide of several metres driven
 *                by surface slopes of 1e-7) FP32 rounding of eta, not the
 *                arithmetic, limits the accuracy; this removes that limit.
 *                8 more bytes per node per step (36 B); one step per pass
 *                with ordinary launches (tblock 2 and persistent are accepted
 *                and run as one-step graph / stream launches).  The
 *                free surface extrapolated onto a DISCHARGE edge is rounded
 *                to FP32 (its low part is 0).  Switching it on sets the low
 *                parts to 0 (switching either way copies the state into the second
 *                buffer set, so the next residual is 0); mlb_set_state splits
 *                h - H exactly into the
 *                pair, mlb_get_state returns H + high + low,
 *                mlb_set_state_device sets the low parts to 0 and
 *                mlb_get_state_device returns the high part.
 * MLB_E_STATE if the grid belongs to a live batch.  The grids of a batch must
 * share the mode (mlb_batch_create: MLB_E_INVAL otherwise); the warm start
 * (mlb_net_infer, mlb_warm_start_run) takes FP32 grids only. */
enum { MLB_SURFACE_FP32 = 0, MLB_SURFACE_COMPENSATED = 1 };
mlb_status mlb_set_surface(mlb_grid* g, int32_t mode);

/* Uniform wind speed (u_wx, u_wy) [m/s]: tau_w / rho = rho_air c_w u_w |u_w| / rho_w
 * (Eq. wind_u-stress). */
mlb_status mlb_set_wind(mlb_grid* g, double uwx, double uwy);
/* Uniform wind stress divided by the water density [m^2/s^2]. */
mlb_status mlb_set_wind_stress(mlb_grid* g, double tx_over_rho, double ty_over_rho);
/* Chezy coefficient: C_b = g / cz^2 (Eq. bed-stress); cz <= 0 removes friction. */
mlb_status mlb_set_chezy(mlb_grid* g, double cz);
/* DEPTH edge data: h = h_mean + amp - amp sin(2 pi t / period + phase);
 * period <= 0 means the constant h_mean + amp - amp sin(phase).
 * MLB_E_INVAL unless the edge is of kind DEPTH. */
mlb_status mlb_set_edge_depth(mlb_grid* g, int edge, double h_mean, double amp,
                              double period, double phase);
/* DISCHARGE edge data (hu, hv) [m^2/s]; MLB_E_INVAL unless the edge is DISCHARGE. */
mlb_status mlb_set_edge_discharge(mlb_grid* g, int edge, double qx, double qy);

/* State from host arrays h, hu, hv [ny][ld] (copied; eta = h - H is rounded
 * to FP32).  Any of hu / hv may be NULL (zero).  Resets the step counter to
 * step0 (t = step0 dt). */
mlb_status mlb_set_state(mlb_grid* g, const double* h, const double* hu, const double* hv,
                         int64_t ld, int64_t step0);
/* State from device FP32 arrays eta, qx, qy, each [ny][nx] contiguous
 * (device-to-device copy on the context stream; the step counter is kept). */
mlb_status mlb_set_state_device(mlb_grid* g, const float* eta, const float* qx, const float* qy);
/* Current h = H + eta, hu, hv into host arrays [ny][ld] (any may be NULL);
 * synchronises the stream.  MLB_E_DEVICE if a persistent launch of the grid
 * gave up at a pass barrier (its passes are incomplete; set the state again). */
mlb_status mlb_get_state(mlb_grid* g, double* h, double* hu, double* hv, int64_t ld);
/* Current FP32 fields copied to device arrays [ny][nx] (any may be NULL).
 * Enqueued; it waits for the stream only after a persistent launch, to report
 * a give-up at a pass barrier (MLB_E_DEVICE). */
mlb_status mlb_get_state_device(mlb_grid* g, float* eta, float* qx, float* qy, float* H);

/* Advances nsteps steps (enqueued on the context stream; returns without
 * waiting).  The call's last pass is a checked one: it also reduces its last
 * step into the FP64 diagnostic sums of the grid (the residual against the
 * step before, which a two-step pass holds in registers), kept with the grid
 * for mlb_diag.  With two steps per pass an odd count starts with one single
 * step.  MLB_E_STATE if the grid belongs to a live batch; MLB_E_DEVICE if an
 * earlier persistent launch of the grid gave up at a pass barrier. */
mlb_status mlb_step(mlb_grid* g, int64_t nsteps);
/* Diagnostics of the last step (a9: FP64 mass, residual, max speed and
 * non-finite count): those the last checked pass kept, or, when the fields
 * were set since (set_state*, set_bathymetry, set_mask, set_surface,
 * mlb_net_infer; both buffers then hold the state), one reduction pass over
 * the state, whose residual is 0.  Syncs.  MLB_E_DEVICE if a persistent launch
 * gave up at a pass barrier. */
mlb_status mlb_diag(mlb_grid* g, mlb_diag_t* out);
/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): mlb_diag
 * with the result written to out_dev, an mlb_diag_t in device memory,
 * enqueued on the context stream without waiting; it never builds the grid's
 * launch plan and allocates nothing.  When the fields were set since the last
 * checked pass it reduces the state with partial sums of tiles of 64 x 64
 * nodes kept in a fixed device array of the library (16384 tiles, 768 KiB
 * per GPU, held until the process ends; each call writes every partial it
 * reads, so nothing needs clearing): MLB_E_INVAL for a grid of more tiles
 * (about 67 M nodes); its sums then equal mlb_diag's to FP64 summation order.
 * Otherwise it takes the sums the last checked pass kept, as mlb_diag does.
 * Calls that overlap on one GPU (several streams or host threads) race on
 * the array.  It does not wait, so it does not report a persistent launch's
 * give-up (mlb_ctx_sync does).  MLB_E_STATE inside a live batch. */
mlb_status mlb_diag_noalloc(mlb_grid* g, mlb_diag_t* out_dev);
/* Steps until the residual of a checked step is <= tol.  Checks every
 * check_every steps (the checked step is reduced in the same kernel pass).
 * MLB_E_NONFINITE on a non-finite value or h <= 0, MLB_E_NOTCONVERGED after
 * max_steps, MLB_E_STALLED under the context's stall rule.  out (may be NULL)
 * receives the last check. */
mlb_status mlb_run_steady(mlb_grid* g, double tol, int64_t max_steps, int32_t check_every,
                          mlb_diag_t* out);

/* Execution options of the step (results are bitwise identical for any
 * choice): rows per tile, temporal block depth (sub-steps per pass), whether
 * step loops are captured and replayed as a hipGraph, and a cap on resident
 * step workgroups per compute unit (fewer concurrent row streams). */
typedef struct {
    int32_t tile_rows;     /* output rows per wave tile, 4..4096                          */
    int32_t tblock;        /* steps per kernel pass: 1, or 2 (temporal blocking: the first
                            * step's level stays in registers; an odd step count takes
                            * one single-step pass first)                                 */
    int32_t use_graph;     /* 1: capture chunks of steps in a hipGraph                    */
    int32_t graph_chunk;   /* steps per captured graph, 2..100000                         */
    int32_t blocks_per_cu; /* 0: no cap; 1..8: at most this many step workgroups per CU   */
    int32_t persistent;    /* 0: one launch per pass (graph chunks).
                            * 1: a call's passes in one cooperative launch with a grid
                            *    barrier between passes, when every tile fits on the device
                            *    at once (else ordinary launches); for small grids, where
                            *    launches dominate.
                            * 2: a call's passes in one persistent launch driven by a
                            *    work queue: a grid of the resident size takes (pass, tile)
                            *    items from an atomic cursor and each item waits for the
                            *    epoch flags of the tiles it depends on, so passes overlap
                            *    instead of draining at a barrier; any grid or batch size.
                            * Waits are bounded: a wait that times out stops the launch;
                            * the next mlb_diag, mlb_run_steady, mlb_get_state*,
                            * mlb_ctx_sync or step call reports MLB_E_DEVICE and the state
                            * must be set again.  The implicit link depth and the
                            * compensated surface take ordinary launches.               */
} mlb_exec_opts;
mlb_status mlb_get_exec_opts(const mlb_grid* g, mlb_exec_opts* o);
mlb_status mlb_set_exec_opts(mlb_grid* g, const mlb_exec_opts* o);

/* Autotuner: times the step for every (tblock, tile_rows, blocks_per_cu)
 * triple of a fixed candidate set (tblock 1 with tile rows 4..45, tblock 2
 * with tile rows 5..44 of the form 3k + 2; caps 0, 2..5), each with graph
 * launches, work-queue launches, and cooperative launches where every tile
 * fits on the device at once, with HIP events (median of 3 runs of `steps`
 * steps; a persistent mode whose first two candidates take more than twice
 * the best graph launch is not timed further), then times the four fastest
 * again (median of 5 runs of at least 200 steps), applies the fastest of
 * those and returns it in *best (may be NULL).  The grid's state and step
 * counter are restored afterwards (results are bitwise independent of these
 * options).  cache_path (may be NULL): a text file of
 * "key tile_rows blocks_per_cu tblock persistent us" lines; a matching key is applied
 * without timing, a new result is appended.  The key holds the device name
 * and the grid shape. */
mlb_status mlb_autotune(mlb_grid* g, int32_t steps, const char* cache_path, mlb_exec_opts* best);

/* Batches: many grids advanced together by one kernel launch per step over a
 * single tile list holding the largest basins first.  Grids keep their
 * own parameters and boundary data; while in a batch they cannot be stepped
 * alone.  Destroying the batch hands the grids back with their state. */
mlb_status mlb_batch_create(mlb_ctx* ctx, mlb_grid* const* grids, int32_t n, mlb_batch** out);
mlb_status mlb_batch_step(mlb_batch* b, int64_t nsteps);
/* Steps the batch until every basin's checked residual is <= tol (per-basin
 * diagnostics in per_basin[n], may be NULL). */
mlb_status mlb_batch_run_steady(mlb_batch* b, double tol, int64_t max_steps,
                                int32_t check_every, mlb_diag_t* per_basin);
mlb_status mlb_batch_set_exec_opts(mlb_batch* b, const mlb_exec_opts* o);
/* As mlb_autotune, for a batch (state of every member restored). */
mlb_status mlb_batch_autotune(mlb_batch* b, int32_t steps, const char* cache_path, mlb_exec_opts* best);
mlb_status mlb_batch_destroy(mlb_batch* b);

/* Kernel time of the last mlb_step / mlb_batch_step call measured with HIP
 * events on the context stream around the step launches [ms]. */
mlb_status mlb_last_step_ms(mlb_ctx* ctx, double* ms);
/* Time per pass of the last call's bulk passes (HIP events on the context
 * stream around them): its passes of `steps_per_pass` steps (the plan's
 * kind, 1 or 2), without a leading single step and without the closing
 * checked pass.  *passes (may be NULL) receives their number.  MLB_E_STATE if
 * the last call had no such pass (fewer than 3 steps with two per pass). */
mlb_status mlb_last_pass_ms(mlb_ctx* ctx, double* ms, int64_t* passes, int32_t* steps_per_pass);

/* Practical HBM bandwidth: copies `bytes` (multiple of 16, >= 4096) between
 * two device buffers the library allocates for the call, `reps` times, with a
 * plain 16-byte-vector copy kernel; returns read + write bytes per second
 * [GB/s] from HIP events.  Used as the reference for measured HBM traffic. */
mlb_status mlb_copy_probe(mlb_ctx* ctx, size_t bytes, int32_t reps, double* gbps);

/* ------------------------------------------------------------------ learned warm start
 * A convolutional encoder-decoder maps a basin's still-water depth and forcing
 * to a guess of its steady state (eta, hu, hv); the step then iterates from the
 * guess (no counterpart in the paper: it only shortens steady-state runs).
 *
 * Architecture (levels L, ch[l] = base_ch 2^l): per encoder level two 3x3
 * convolutions + ReLU (2x2 average pool between levels); per decoder level a
 * nearest x2 upsample, a 3x3 conv + ReLU, concatenation with the encoder
 * level's output, two 3x3 convs + ReLU; a 1x1 head to 3 channels.  The input
 * has in_ch channels (MLB_NET_FEATURES = 8 features, the rest zero):
 *   0  normalised still-water depth H
 *   1, 2  wind stress over density: its direction (unit vector, 0 without
 *         wind) when tau_ref > 0, else normalised tau_x/rho, tau_y/rho
 *   3  normalised |tau|/rho
 *   4  normalised C_b
 *   5, 6  node position x, y mapped to [-1, 1] (the steady surface of a
 *         closed basin depends on where a node lies relative to the walls,
 *         which a finite receptive field cannot see)
 *   7  1 (marks the image edges through the convolutions' zero padding)  Convolutions run on BF16
 * MFMA with FP32 accumulation; FP32 master parameters.  Parameters are ordered
 * layer by layer in forward order, each 3x3 weight [Cout][3][3][Cin] then its
 * bias; the head weight [3][base_ch] then its bias.
 * Requirements: in_ch and base_ch multiples of 32; width / 2^(L-1) a
 * multiple of 32; height a multiple of 2^(L-1); base_ch 2^(L-1) <= 2048. */
typedef struct mlb_net mlb_net;
typedef struct {
    int32_t height, width;   /* field size                                            */
    int32_t in_ch;           /* input channels (>= 6; 6 used)                          */
    int32_t out_ch;          /* 3: eta, hu, hv                                         */
    int32_t base_ch;         /* channels of the finest level                           */
    int32_t levels;          /* >= 2                                                   */
    int32_t max_batch;       /* samples per forward / backward call                    */
} mlb_net_cfg;
#define MLB_NET_FEATURES 8
typedef struct {
    float in_mean[5], in_std[5]; /* H, tau_x/rho, tau_y/rho, |tau|/rho, C_b            */
    float s_eta, s_q;            /* output scales: eta = s_eta f y0, q = s_q f (y1, y2) */
    float tau_ref;               /* > 0: f = |tau|/rho / tau_ref per basin (steady set-up
                                  * and circulation grow with the stress); 0: f = 1    */
} mlb_net_norm;
typedef struct { float lr, beta1, beta2, eps, weight_decay; } mlb_adamw_cfg;

/* Creates a net with He-normal weights from `seed` and zero biases. */
mlb_status mlb_net_create(mlb_ctx* ctx, const mlb_net_cfg* cfg, uint64_t seed, mlb_net** out);
mlb_status mlb_net_destroy(mlb_net* net);
mlb_status mlb_net_param_count(const mlb_net* net, int64_t* n);
/* FP32 parameters to / from host memory (set_params also refreshes the BF16 copies). */
mlb_status mlb_net_get_params(mlb_net* net, float* host, int64_t n);
mlb_status mlb_net_set_params(mlb_net* net, const float* host, int64_t n);
mlb_status mlb_net_set_norm(mlb_net* net, const mlb_net_norm* norm);
mlb_status mlb_net_get_norm(const mlb_net* net, mlb_net_norm* norm);
/* Forward pass: x [n][height][width][MLB_NET_FEATURES] FP32 (device) -> y [n][height][width][3] FP32 (device). */
mlb_status mlb_net_forward(mlb_net* net, const float* x_dev, int32_t n, float* y_dev);
/* Forward + backward of the masked MSE against targets t [n][h][w][3] (device);
 * mask [n][h][w] (device, may be NULL = all ones) with mask_count = its sum.
 * Leaves the parameter gradient in the net (for mlb_net_adamw); *loss (may
 * be NULL) receives the loss; grad_host (may be NULL) receives the gradient. */
mlb_status mlb_net_loss_grad(mlb_net* net, const float* x_dev, const float* t_dev, const float* mask_dev,
                             double mask_count, int32_t n, double* loss, float* grad_host);
/* One AdamW step (decoupled weight decay) with the last gradient. */
mlb_status mlb_net_adamw(mlb_net* net, const mlb_adamw_cfg* cfg);
/* Features of a grid (its still-water depth and forcing, normalised) into
 * x_dev [height][width][MLB_NET_FEATURES]; targets (its current state
 * divided by the output scales; 0 when f = 0) into t_dev [height][width][3].
 * The grid must be height x width. */
mlb_status mlb_net_features(mlb_net* net, mlb_grid* g, float* x_dev);
mlb_status mlb_net_targets(mlb_net* net, mlb_grid* g, float* t_dev);
/* Warm start: writes the net's guess into the grid's state.  The net output
 * is smoothed by the 3x3 binomial filter (edges clamped; it removes
 * grid-scale content the step damps only slowly), its mean surface
 * perturbation is removed so the basin holds its still-water volume (closed
 * basins conserve it, so the steady state has that volume), and discharge
 * is zero on wall nodes.  MLB_E_STATE for a grid with a node mask (the net
 * knows rectangular basins only; the same holds for mlb_warm_start_run). */
mlb_status mlb_net_infer(mlb_net* net, mlb_grid* g);
mlb_status mlb_net_save(const mlb_net* net, const char* path);
mlb_status mlb_net_load(mlb_net* net, const char* path);

/* Training over a dataset resident in device memory: x [n][height][width][MLB_NET_FEATURES],
 * t [n][height][width][3], optional mask [n][height][width] (NULL = all ones).
 * Each epoch visits the samples in a fresh random order (seeded) in
 * minibatches of `batch` (the last, smaller one included); each minibatch is
 * one mlb_net_loss_grad + one AdamW step.  Step size: linear ramp over
 * warmup_steps, then cosine decay from lr to lr_min over the remaining steps.
 * epoch_loss (host, may be NULL) receives the mean minibatch loss of each
 * epoch.  The AdamW moments continue from earlier calls. */
typedef struct {
    int32_t epochs;
    int32_t batch;           /* 1 .. max_batch                                         */
    float lr, lr_min;
    int32_t warmup_steps;
    float beta1, beta2, eps, weight_decay;
    uint64_t seed;
} mlb_train_cfg;
mlb_status mlb_net_train(mlb_net* net, const float* x_dev, const float* t_dev, const float* mask_dev, int32_t n,
                         const mlb_train_cfg* cfg, double* epoch_loss);

/* Warm-started steady-state run of a closed or open basin: the grid's current
 * state is the cold start.  Steps:
 *   1. one probe step from the cold start gives its first residual r0_cold;
 *   2. mlb_net_infer writes the net's guess (mean surface removed, walls
 *      q = 0); its first step gives r0_guess;
 *   3. the run continues from the guess like mlb_run_steady, unless the guess
 *      is non-finite, r0_guess > r0_cold, or the residual rose at 3
 *      consecutive checks and exceeds its value at the first check (or a
 *      non-finite value appears): then the cold start is restored (fields and
 *      step counter) and run with mlb_run_steady;
 *   4. on convergence, guess_err receives the relative L2 distance of the
 *      guess to the converged state per field (eta, hu, hv).
 * A stall (mlb_set_stall_checks) of the run from the guess is not a
 * fallback: the guess led to the same steady state, held at FP32's floor.
 * Returns MLB_OK when converged, else the status of the last run. */
typedef enum {
    MLB_WARM_NONE = 0,            /* the guess was used                              */
    MLB_WARM_NONFINITE_GUESS = 1, /* non-finite or dry guess                         */
    MLB_WARM_WORSE_THAN_COLD = 2, /* r0_guess > r0_cold                              */
    MLB_WARM_DIVERGING = 3        /* residual rising or non-finite while running     */
} mlb_warm_fallback;
typedef struct {
    int32_t used_guess;      /* 1: converged from the guess; 0: from the cold start     */
    int32_t fallback;        /* mlb_warm_fallback                                       */
    double r0_guess, r0_cold;
    double infer_ms;         /* features + forward + projection (HIP events)            */
    double wall_s;           /* the whole call, host clock                              */
    int64_t steps;           /* steps of the run that converged                         */
    int64_t steps_total;     /* all steps: probe, abandoned warm steps, final run       */
    double guess_err[3];     /* relative L2 of the guess vs the converged state         */
    mlb_diag_t diag;         /* diagnostics at the end                                  */
} mlb_warm_report;
mlb_status mlb_warm_start_run(mlb_grid* g, mlb_net* net, double tol, int64_t max_steps, int32_t check_every,
                              mlb_warm_report* report);

/* ------------------------------------------------------------- eLABSWE baseline
 * The lattice Boltzmann equation the method is derived from (Eq. lb.1): nine
 * stored distributions per node, relaxed with a single time tau > 1/2 and
 * streamed (pull form, Eq. lb.Mac.1), f_a^eq of Eq. feq-full, the link depth
 * of Eq. h-bar and the link-midpoint force; viscosity
 * nu = e^2 dt (2 tau - 1) / 6 (Eq. viscosity) with the grid's e and dt (so
 * tau = 1 is the grid's own nu, and the step is then the streaming-only one).
 * Bounced links take the node's own post-collision f*_abar; nodes on wall
 * edges and WALL nodes end each step at f^eq(h', 0); SOLID nodes keep their
 * distributions.  A baseline for measuring what stored distributions cost
 * (72 B per node moved per step against 28 B); it has no diagnostics,
 * graphs or batches.
 *
 * mlb_elab_create takes the grid's bed, node mask, edges (WALL / PERIODIC
 * only: MLB_E_INVAL otherwise), forcing and tile rows as they are at the call,
 * and starts from f = f^eq of the grid's current state.  The grid must
 * outlive the baseline (mlb_grid_destroy returns MLB_E_STATE meanwhile) and
 * must use Eq. h-bar.  Device memory: 21 planes of nx * ny floats (with the
 * grid's pitch), allocated by the library.
 * mlb_elab_step enqueues nsteps steps (timed by mlb_last_step_ms).
 * mlb_elab_get_state: h = H + (sum f - H), hu, hv into host arrays [ny][ld]
 * (synchronises); mlb_elab_get_dist_device: the distributions as
 * [9][ny][nx] FP32 into a device array (enqueued on the stream). */
typedef struct mlb_elab mlb_elab;
mlb_status mlb_elab_create(mlb_grid* g, double tau, mlb_elab** out);
mlb_status mlb_elab_step(mlb_elab* s, int64_t nsteps);
mlb_status mlb_elab_get_state(mlb_elab* s, double* h, double* hu, double* hv, int64_t ld);
mlb_status mlb_elab_get_dist_device(mlb_elab* s, float* f);
mlb_status mlb_elab_destroy(mlb_elab* s);

#ifdef __cplusplus
}
#endif
#endif /* MLB_H */
