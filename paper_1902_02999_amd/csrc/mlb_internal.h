// Internal data structures shared by the gfx950 kernels and the host runtime.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mlb {

// Output columns per wave strip: a wave's 64 lanes cover columns x0-1 .. x0+62;
// lanes 1..62 produce outputs, lanes 0 and 63 only supply neighbour values.
constexpr int kStripOut = 62;
// Two steps per pass: lanes 0..63 cover x0-2 .. x0+61, lanes 2..61 produce outputs.
constexpr int kStripOut2 = 60;
constexpr int kWave = 64;
constexpr int kBlock = 256;            // 4 independent waves per workgroup
constexpr int kPartials = 6;           // per-tile FP64 partial sums

enum { EDGE_WALL = 0, EDGE_PERIODIC = 1, EDGE_DEPTH = 2, EDGE_DISCHARGE = 3 };
// Node kinds of the optional geometry mask.
enum { NODE_FLUID = 0, NODE_WALL = 1, NODE_SOLID = 2 };
// TileDev::flags
enum { TILE_MASKED = 1 };   // the tile's window holds a WALL or SOLID node

// Per-basin descriptor read by the step kernel (device memory).
struct BasinDev {
    float* eta[2];
    float* qx[2];
    float* qy[2];
    const float* H;
    const uint8_t* mask;   // node kinds (pitch ld bytes) or nullptr
    // implicit link depth: per-node 1/(1+kappa), kappa_x, kappa_y planes
    // (pitch ld floats), nullptr for the old-time link depth
    const float* cw;
    const float* ckx;
    const float* cky;
    // compensated surface: low part of eta per buffer (nullptr: plain FP32)
    float* etal[2];
    int64_t* stepc;        // [2]: step counter, read from [rd], written to [1-rd]
    double* dres;          // [8]: the basin's last finalised diagnostics (grid header), or nullptr
    int32_t nx, ny, ld;
    int32_t swap;          // buffer read by a launch of parity p is p ^ swap
    int32_t per_x, per_y;
    int32_t kind[4];       // W, E, S, N
    int32_t extrap;        // 1 or 2
    int32_t first_tile, ntiles;     // in the one-step tile list
    int32_t first_tile2, ntiles2;   // in the two-step tile list
    // FP32 constants of the step (computed in FP64 on the host, then rounded)
    float e;               // lattice speed
    float tpx, tpy;        // (dt/2) tau_w / rho
    float cfr;             // (dt/2) C_b
    float omh;             // (dt/2) Omega
    float c3e;             // 1 / (3e)
    float ckk;             // 2 / (3e^2)
    float c6, c12, c4;     // 1/(6e^2), 1/(12e^2), 1/(4e^2)
    float cma, cmd;        // g/(6e^2), g/(24e^2)
    float cqa, cqd;        // g/(6e),  g/(24e)
    float bc_qx[4], bc_qy[4];
    double dt;
    double bc_hmean[4], bc_amp[4], bc_om[4], bc_phase[4];
};

// Grid barrier state of persistent launches (device memory, zeroed once).
struct SyncState {
    uint64_t count;        // arrivals, accumulated over launches
    int32_t err;           // set when a bounded wait gave up
    int32_t pad;
};

// Work queue of a persistent launch (device memory).  Items are (pass, tile)
// in pass-major, list order; a wave takes the next item from the cursor and
// waits until every tile its item depends on (the tiles whose owned nodes
// its window reads, and those whose windows read its owned nodes) has
// completed the previous pass.
struct WorkQueue {
    uint32_t* cursor;        // [1] items handed out in the current launch
    uint32_t* epoch;         // [ntiles] passes each tile has completed, over all launches
    const int32_t* nbr_off;  // [ntiles + 1] dependency list of tile t: nbr[nbr_off[t] .. nbr_off[t+1])
    const int32_t* nbr;      // tile indices (the tile itself included), at most 64 per tile
    int64_t* base;           // [nbasins] each basin's step counter when the launch starts
    int32_t* err;            // set when a bounded wait gave up (the plan's SyncState::err)
};

// One wave's work item: a strip of up to 62 columns and `rows` rows.
struct TileDev {
    int32_t basin;
    int32_t x0, y0, rows;  // first output column / row and number of rows computed
    int32_t xo, yo;        // first owned column / row (overlapped edge tiles store only these)
    int32_t flags;         // TILE_*
    int32_t pad;
};

// eLABSWE baseline (elab_kernels.hip): nine planes per buffer of the
// distributions minus the node's still-water equilibrium, [9][ny][ld]
// floats, plane = ld * ny rounded up (floats between planes).
struct ElabDev {
    float* f[2];
    const float* H;
    const uint8_t* mask;   // node kinds or nullptr
    int64_t plane;
    int32_t nx, ny, ld;
    int32_t per_x, per_y;
    // FP32 constants (computed in FP64 on the host)
    float e;               // lattice speed
    float tx, ty, cb, om;  // tau_w / rho, C_b, Omega
    float cfp;             // dt / (2e)
    float g6, c6, c3, c2;  // g/(6e^2), 1/(6e^2), 1/(3e), 1/(2e^2)
    float gb;              // g/(2e^2)
    float rtau;            // 1 / tau
};

hipError_t launch_elab_step(const ElabDev& D, const TileDev* d_tiles, int ntiles, int rd, hipStream_t s);
hipError_t launch_elab_init(const ElabDev& D, const float* eta, const float* qx, const float* qy, hipStream_t s);
hipError_t launch_elab_macro(const ElabDev& D, int rd, float* eta, float* qx, float* qy, hipStream_t s);
hipError_t launch_elab_dist(const ElabDev& D, int rd, float* out, hipStream_t s);

// Host-side launchers (mlb_kernels.hip).
// tblock 1: one step, tblock 2: two steps over tiles of kStripOut2 columns;
// diag: the (last) step is reduced into the tile partials.  masked: the tile list may hold
// TILE_MASKED tiles; implicit: every basin has the implicit link-depth
// planes; comp: every basin has a compensated surface (one step only);
// closed: no basin has an open (DEPTH or DISCHARGE) edge, so the two-step
// kernel is the one without the open-edge logic.
hipError_t launch_step(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity,
                       double* d_partials, int diag, int tblock, int masked, int implicit, int comp, int closed,
                       unsigned dyn_lds, hipStream_t s);
// The two-step kernels (mlb_kernels2.hip); launch_step forwards tblock 2 here.
hipError_t launch_step2(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity,
                        double* d_partials, int diag, int masked, int implicit, int closed, unsigned dyn_lds,
                        hipStream_t s);
// npasses passes of `kind` steps in one cooperative launch (all tiles
// resident); base = sync->count at launch.  Fails (no launch) when the grid
// cannot be co-resident.
hipError_t launch_persistent(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles, int parity0,
                             int npasses, int kind, int masked, SyncState* sync, uint64_t base, int spin_limit,
                             hipStream_t s);
// Workgroups of the persistent kernel that fit on the device at once.
int persistent_capacity(int kind, int masked, int ncu);
// npasses passes of `kind` steps in one launch of `nblocks` workgroups driven
// by the work queue q (the cursor is reset and the basins' step counters
// snapshot by a prologue kernel on the same stream).  epoch0: passes the
// queue's tiles completed before this launch.  closed: no basin has an open
// edge (two-step passes take the kernel without open-edge logic).
hipError_t launch_workqueue(const BasinDev* d_basins, int nbasins, const TileDev* d_tiles, int ntiles, int parity0,
                            int npasses, int kind, int masked, int closed, const WorkQueue& q, uint32_t epoch0,
                            int spin_limit, int nblocks, unsigned dyn_lds, hipStream_t s);
// Resident workgroups per CU of the work-queue kernel.
int workqueue_occupancy(int kind, int masked, int closed);
hipError_t launch_reduce_state(const BasinDev* d_basins, const TileDev* d_tiles, int ntiles,
                               int parity, double* d_partials, hipStream_t s);
int step_occupancy(int diag);
hipError_t launch_copy_probe(const void* src, void* dst, size_t bytes, int nblocks, hipStream_t s);
// Per-basin sums of the tile partials of a pass of `kind` steps (1 also for the
// state reduction) into d_out[8 * basin] and each basin's result slot.
hipError_t launch_finalize(const BasinDev* d_basins, int nbasins, const double* d_partials,
                           double* d_out, int kind, hipStream_t s);

}  // namespace mlb
