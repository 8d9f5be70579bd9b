// Runtime objects shared by the host-side translation units of libmlb.so.
#pragma once

#include <string>
#include <vector>

#include "../../include/mlb.h"
#include "mlb_internal.h"

namespace mlb {

// Sets the calling thread's last error message and returns s.
mlb_status fail(mlb_status s, const std::string& msg);

// Stall rule of steady-state runs: it counts checks without a new lowest
// residual only once that lowest residual is within this factor of the
// tolerance (a run from rest passes through transient minima far above it).
constexpr double kStallBand = 10.0;

// Looks up the device's copy of the allocation-free entry point's scratch
// array (mlb_noalloc.hip); once per device, with the device current.
mlb_status noalloc_setup(int device);

// Sets a grid's step counter (host and device copies); syncs the stream.
mlb_status grid_set_step(mlb_grid* g, int64_t s);

// One-step wave tiles of a grid (mask classification included).
void grid_tiles(const mlb_grid* g, int rows, std::vector<TileDev>& out);

}  // namespace mlb

#define HIPCHK(call)                                                                        \
    do {                                                                                    \
        hipError_t e_ = (call);                                                             \
        if (e_ != hipSuccess)                                                               \
            return ::mlb::fail(e_ == hipErrorOutOfMemory ? MLB_E_NOMEM : MLB_E_DEVICE,      \
                               std::string(#call) + ": " + hipGetErrorString(e_));          \
    } while (0)

#define CHK(expr)                                 \
    do {                                          \
        mlb_status s_ = (expr);                   \
        if (s_ != MLB_OK) return s_;              \
    } while (0)

namespace mlb {

struct Plan;
// Takes a plan off its context's list of plans with an unchecked persistent launch.
void plan_unwatch(Plan& P);
// The grid's fields were replaced: its last checked diagnostics no longer apply.
void grid_state_changed(mlb_grid* g);

// Work queue of one tile list of a plan (device buffers, built on first use
// by a work-queue launch; see WorkQueue).
struct WqBuf {
    WorkQueue q{};
    uint32_t passes = 0;     // passes its tiles have completed (epoch0 of the next launch)
    bool ok = false;         // built
    bool failed = false;     // a tile has more than 64 dependencies: ordinary launches
    void release()
    {
        (void)hipFree(q.cursor); (void)hipFree(q.epoch); (void)hipFree((void*)q.nbr_off);
        (void)hipFree((void*)q.nbr); (void)hipFree(q.base);
        q = WorkQueue{};
        passes = 0; ok = false; failed = false;
    }
};

// Device-side plan of a set of basins: descriptors, tile list,
// reduction partials, and an optional captured chunk of steps.
struct Plan {
    std::vector<BasinDev> hb;
    std::vector<TileDev> ht;       // one step per pass
    std::vector<TileDev> ht2;      // two steps per pass (empty unless tblock 2)
    BasinDev* db = nullptr;
    TileDev* dt = nullptr;
    TileDev* dt2 = nullptr;
    double* dpart = nullptr;
    double* dout = nullptr;
    double* hout = nullptr;  // pinned
    int parity = 0;
    hipGraphExec_t gexec = nullptr;
    hipGraph_t graph = nullptr;
    int gparity = -1;
    int gsteps = 0;
    int gkind = 0;             // steps per launch in the captured graph
    SyncState* dsync = nullptr;  // grid barrier state of persistent launches
    int32_t* herr = nullptr;     // pinned copy of dsync->err
    uint64_t sync_base = 0;      // dsync->count when the next persistent launch starts
    bool coop_failed = false;    // a persistent launch was refused: use ordinary ones
    WqBuf wq[2];                 // work queues of the one-step [0] and two-step [1] tile lists
    bool err_pending = false;    // herr holds a stream-ordered copy of dsync->err not yet checked
    mlb_ctx* watch = nullptr;    // the context listing this plan while err_pending
    unsigned gdyn = 0;         // dynamic LDS the captured graph was launched with
    bool masked = false;       // some basin has a node mask: one-step passes, masked kernel
    bool implicit = false;     // the basins use the implicit link depth: one-step passes
    bool comp = false;         // the basins have a compensated surface: one-step passes
    bool closed = false;       // no basin has an open edge: the two-step kernel without open-edge logic
    bool built = false;

    void release()
    {
        plan_unwatch(*this);
        if (gexec) (void)hipGraphExecDestroy(gexec);
        if (graph) (void)hipGraphDestroy(graph);
        gexec = nullptr; graph = nullptr; gparity = -1; gsteps = 0; gkind = 0;
        (void)hipFree(db); (void)hipFree(dt); (void)hipFree(dt2); (void)hipFree(dpart);
        (void)hipFree(dsync);
        wq[0].release(); wq[1].release();
        if (herr) (void)hipHostFree(herr);
        dsync = nullptr; herr = nullptr; sync_base = 0; coop_failed = false; err_pending = false;
        (void)hipFree(dout);
        if (hout) (void)hipHostFree(hout);
        db = nullptr; dt = nullptr; dt2 = nullptr; dpart = nullptr; dout = nullptr; hout = nullptr;
        built = false;
    }
};

}  // namespace mlb

struct mlb_ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    int live = 0;
    int ncu = 0;
    int lds_per_cu = 0;        // bytes
    std::string arch;          // gcnArchName, for autotuner cache keys
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    bool timed = false;
    // the last call's bulk passes (its passes of the plan's kind, without a
    // leading single step and the closing checked pass), timed alone
    hipEvent_t ev2 = nullptr, ev3 = nullptr;
    int64_t bulk_passes = 0;
    int bulk_kind = 0;
    std::vector<mlb::Plan*> watch;   // plans with an unchecked persistent launch
    int stall_checks = 0;      // 0: off
    int spin_limit = 1 << 22;  // polls of a persistent launch's barrier wait (MLB_SPIN_LIMIT)
};

struct mlb_grid {
    mlb_ctx* ctx = nullptr;
    mlb_params p{};
    int ld = 0;
    size_t plane = 0;          // floats per field plane
    char* base = nullptr;
    bool own = false;
    float* eta[2] = {nullptr, nullptr};
    float* qx[2] = {nullptr, nullptr};
    float* qy[2] = {nullptr, nullptr};
    float* H = nullptr;
    int64_t* stepc = nullptr;
    double* dres = nullptr;    // [8] in the workspace header: the last checked pass's finalised sums
    bool diag_fresh = false;   // dres holds the diagnostics of the current state's last step
    std::vector<float> Hf;     // stored (FP32) still-water depth, host copy
    std::vector<double> Hd;    // still-water depth zeta_ref - z_b as given (FP64):
                               // host conversions h <-> eta and the mass use it
    uint8_t* dmask = nullptr;  // node kinds on the device (pitch ld bytes), or none
    std::vector<uint8_t> hmask;  // host copy (pitch ld), empty without a mask
    int hbar = MLB_HBAR_SEMI_IMPLICIT;
    float* dcoef = nullptr;    // implicit link depth: 3 planes (1/(1+kappa), kappa_x, kappa_y)
    float* etal = nullptr;     // compensated surface: low part of eta, 2 planes (one per buffer)
    int cur = 0;
    int64_t step = 0;
    double e = 0, dt = 0, sumH = 0, Hmax = 0;
    double tx = 0, ty = 0, cb = 0;
    double bc_hmean[4] = {0, 0, 0, 0}, bc_amp[4] = {0, 0, 0, 0}, bc_om[4] = {0, 0, 0, 0},
           bc_phase[4] = {0, 0, 0, 0}, bc_qx[4] = {0, 0, 0, 0}, bc_qy[4] = {0, 0, 0, 0};
    mlb_batch* batch = nullptr;
    mlb_exec_opts opts{15, 1, 1, 64, 3, 0};
    mlb::Plan plan;
    int elab_refs = 0;         // live eLABSWE baselines built on this grid
    bool dirty = true;         // descriptor must be re-uploaded
    bool stale_plan = true;    // tiles / allocation must be rebuilt
};

struct mlb_batch {
    mlb_ctx* ctx = nullptr;
    std::vector<mlb_grid*> grids;
    mlb_exec_opts opts{15, 1, 1, 64, 3, 0};
    mlb::Plan plan;
    bool stale_plan = true;
};

