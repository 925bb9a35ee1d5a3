// Plan object of the gfx950 multigrid library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/vmg.h"
#include "vmg_internal.h"

#ifndef VMG_FOLD_PROLONG
#define VMG_FOLD_PROLONG true
#endif

namespace vmg {

struct LevelBuf {
    Geom g;
    double* phi[2] = {nullptr, nullptr};   // ping-pong pair (sweeps read one, write the other)
    double* phiold = nullptr;              // R phi^h kept for the correction (coarse levels)
    double* f = nullptr;                   // FAS right-hand side (level 0: caller's source)
    double* delta = nullptr;
    double* rd = nullptr;                  // R d^h (coarse levels)
    LevelScalars* sc = nullptr;            // device scalars (cbar)
    int cur = 0;                           // which phi[] holds the current iterate
    // mixed path (FP32 correction problem)
    float* e[2] = {nullptr, nullptr};      // correction, ping-pong
    float* eold = nullptr;                 // R e^h (coarse levels)
    float* r = nullptr;                    // inner right-hand side (level 0: -d)
    float* pt = nullptr;                   // FP32 base state phi~
    float* t0 = nullptr;                   // +-sqrt|D0| of the base state
    float* rdf = nullptr;                  // R d_e (coarse levels)
    LevelScalars* scf = nullptr;           // inner cbar
    int ecur = 0;
};

struct GridState {
    vmg_grid desc;
    std::vector<LevelBuf> lev;
    NormOut* norm_dev = nullptr;
};

// One level of a batch of Dirichlet grids: pooled buffers shared by every grid
// that has this level, plus the device work lists of the batched kernels.
struct BatchLevel {
    std::vector<int> members;        // grid ids with a level here, in id order
    std::vector<int> coarsest;       // per member: 1 if this is its coarsest level
    int64_t pool = 0;                // elements per pooled buffer
    double* phi[2] = {nullptr, nullptr};
    double *phiold = nullptr, *f = nullptr, *delta = nullptr, *rd = nullptr;
    float* e[2] = {nullptr, nullptr};
    float *eold = nullptr, *r = nullptr, *pt = nullptr, *t0 = nullptr, *rdf = nullptr;
    LevelScalars* sc = nullptr;      // one per member
    LevelScalars* scf = nullptr;
    Geom* d_geom = nullptr;          // member geometries at this level
    Geom* d_geom_fine = nullptr;     // same grids one level finer (levels >= 1)
    Geom* d_geomC = nullptr;         // members whose coarsest level is this one
    int nC = 0;
    int4* d_sitems = nullptr;        // smoother work list (members that continue below)
    int nsitems = 0;
    int2* d_cells = nullptr;         // 256-cell blocks of every member at this level
    int ncells = 0;
    int2* d_store = nullptr;         // 256-element blocks of each member's padded storage (levels >= 1)
    int nstore_items = 0;
    SmoothCfg cfg{8, 16};            // schedule of the persistent smoother on this level
    int2* d_ghosts = nullptr;        // 256-value blocks of each member's ghost shell (levels >= 1)
    int nghost_items = 0;
    int64_t cells_A = 0, cells_C = 0;
    int cur = 0, ecur = 0;
};

struct Plan {
    std::vector<GridState> grids;
    vmg_params params;
    Coef coef;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;      // created when the caller passes stream 0
    SmoothCfg cfg;                         // finest-level schedule of the fused sweep
    std::vector<SmoothCfg> lcfg;           // tuned schedules of levels >= 1 (empty: level_cfg rule)
    int nu1 = 2, nu2 = 2, ncoarse = 40;
    int inner = 2;                         // mixed: FP32 inner V-cycles per outer iteration
    int nu1c = 0, nu2c = 0;                // sweeps below the finest level (0, 0: nu1, nu2)
    bool use_tail = true;                  // periodic coarse levels <= TAIL_CELLS in one launch
    bool fold_prolong = VMG_FOLD_PROLONG;  // periodic: prolongation folded into the first post-sweep
    int batch_blocks = 1024;               // blocks of a batched plan's persistent smoother launch
    bool periodic = true;
    bool mixed = false;
    bool has_source = false;
    bool solved = false;
    double* partials = nullptr;
    double* partials_b = nullptr;          // second set (coarse right-hand-side pass)
    NormOut* host_norm = nullptr;          // pinned
    // replayable iterations, one per (source given, finest-level ping-pong parity);
    // all four are captured when the plan is created (VMG_GRAPH)
    hipGraphExec_t graph[2][2];
    bool graph_ok[2][2] = {{false, false}, {false, false}};
    int64_t graph_updates[2][2] = {{0, 0}, {0, 0}};   // cell updates / finest sweeps of one replay
    int64_t graph_finest[2][2] = {{0, 0}, {0, 0}};
    bool graph_flip[2][2] = {{false, false}, {false, false}};   // replay moves the finest phi
    int64_t cell_updates = 0, finest_sweeps = 0;
    std::vector<void*> allocs;
    // finest-sweep timing (vmg_plan_time_sweeps): event pairs around every
    // finest-level sweep launched by a solve, also recorded into the graphs
    bool time_sweeps = false;
    bool timing_active = false;            // inside a solve or a graph capture
    std::vector<hipEvent_t> tev;           // [2i] before, [2i+1] after run i of consecutive sweeps
    std::vector<int> tev_count;            // sweeps in run i
    int tev_used = 0;                      // pairs recorded since the last collection
    int graph_tev[2][2] = {{0, 0}, {0, 0}};
    double sweep_us = 0.0;
    int64_t sweep_n = 0;
    // per-level timing (vmg_plan_time_levels): event pairs around the work of
    // each level of a cycle (head: pre-sweeps, restriction, coarse rhs; tail:
    // prolongation, post-sweeps; the coarse tail / coarsest solve as one piece at
    // its top level), tagged with the level; solves then launch directly
    bool time_levels = false;
    std::vector<hipEvent_t> lev_ev;        // [2i] before, [2i+1] after piece i
    std::vector<int> lev_tag;              // level of piece i
    int lev_used = 0;
    std::vector<double> level_us;          // summed per level since enabled
    int64_t level_cycles = 0;              // iterations timed since enabled
    // residual history of the last solve (vmg_plan_history): per grid, the
    // norms before the first iteration and after each one
    std::vector<std::vector<vmg_history>> history;
    // batched Dirichlet plans
    bool tuned_from_cache = false;
    struct TuneEntry { int level; SmoothCfg cfg; double us; };
    std::vector<TuneEntry> tune_log;       // autotuner timings (one sweep of a level, us)
    bool batched = false;
    std::vector<BatchLevel> blev;
    int64_t* d_uoff = nullptr;       // caller offsets of each grid's cells
    int64_t* d_goff = nullptr;       // caller offsets of each grid's ghosts
    int2* d_gitems = nullptr;        // 256-value blocks of every grid's ghosts
    int bngitems = 0;
    int* d_first = nullptr;          // first norm block of each grid (+ end)
    int* d_first1 = nullptr;         // the same for level 1 (tau^h), when every grid has it
    NormOut* d_norms = nullptr;
};

vmg_status fail(vmg_status st, const std::string& msg);
// bracket a run of `launches` consecutive finest-level sweeps with timing
// events (no-op unless enabled)
// pre- and post-smoothing sweeps of level l (the finest level runs nu1/nu2, the
// coarser ones nu1c/nu2c when those are set)
inline int pre_sweeps(const Plan* P, int l) { return l > 0 && (P->nu1c | P->nu2c) ? P->nu1c : P->nu1; }
inline int post_sweeps(const Plan* P, int l) { return l > 0 && (P->nu1c | P->nu2c) ? P->nu2c : P->nu2; }
hipError_t sweep_mark(Plan* P, bool begin, int launches);
// bracket the work of level l (begin / end) when per-level timing is on
hipError_t level_mark(Plan* P, int l, bool begin);
CoefF make_coef_f(const Coef& c, double h);
vmg_status alloc_mixed(Plan* P);
hipError_t enqueue_outer(Plan* P);          // one mixed-precision outer iteration (+ norms to host)
hipError_t mixed_initial_pass(Plan* P);     // cast pass of the initial guess (+ norms to host)
hipError_t mixed_prepare(Plan* P);          // per-solve set-up of the FP32 ghost shells
hipError_t smooth_corr_level(Plan* P, GridState& G, int l, bool zero_in = false, const ProlongInF* pro = nullptr);
hipError_t smooth_corr_level_n(Plan* P, GridState& G, int l, int count, bool zero_in = false,
                               const ProlongInF* pro = nullptr);
// coarse-correction prolongation + nu2 post-sweeps of level l (FP64 / correction)
hipError_t post_smooth(Plan* P, GridState& G, int l, int nu2);
hipError_t post_smooth_corr(Plan* P, GridState& G, int l, int nu2);
vmg_status build_batch(Plan* P);
vmg_status autotune(Plan* P);
// levels of a plan that run the fused sweep (the levels a schedule applies to)
int swept_level_count(const Plan* P);
// (re)record the replayable iterations of a VMG_GRAPH plan (no-op without the flag)
vmg_status capture_graphs(Plan* P);
// cycle schedule of a plan (nu1, nu2, inner cycles, coarsest sweeps, coarse tail,
// persistent launch size); set_cycle validates, installs and re-records graphs
void get_cycle(const Plan* P, vmg_cycle* c);
vmg_status set_cycle(Plan* P, const vmg_cycle* c);
// cached cycle schedule for this plan's key, if the tuning cache holds one
bool cached_cycle(const Plan* P, vmg_cycle* c);
vmg_status tune_cycle(Plan* P, const double* delta, const double* ghost, const double* source, double* phi_work,
                      vmg_cycle* best, double* best_ms);
vmg_status solve(Plan* P, const double* delta, const double* ghost, const double* source, double* phi,
                 vmg_result* out);
// `count` FP64 sweeps of level l (in pairs on the brick schedule)
hipError_t smooth_level_public(Plan* P, GridState& G, int l, int count);
// whether the first post-sweep of level l (schedule cfg) takes the prolongation
// from coarse level gc
bool fold_prolong_here(const Plan* P, const Geom& g, const Geom& gc, const SmoothCfg& cfg);
// schedule of the fused sweep on level l of a single-grid (periodic) plan
SmoothCfg level_schedule(const Plan* P, int l, const Geom& g);
// first level handled by the periodic coarse tail (FP64 plans), or -1
int tail_level(const Plan* P, const GridState& G);
// batched plans: rebuild the persistent smoother's work list of level l for cfg;
// one sweep of every grid on level l
hipError_t batch_set_level_cfg(Plan* P, int l, SmoothCfg cfg);
hipError_t batch_smooth_level(Plan* P, int l);
int64_t batch_partials_needed(const Plan* P);
hipError_t batch_build_smooth_items(Plan* P);
hipError_t batch_enqueue_iteration(Plan* P);
hipError_t batch_check_delta(Plan* P, const double* delta);
hipError_t batch_setup(Plan* P, const double* delta, const double* ghost, const double* source, const double* phi);
hipError_t batch_outputs(Plan* P, double* phi);
hipError_t batch_smooth_finest(Plan* P);
int batch_parity(const Plan* P);
void batch_flip_parity(Plan* P);
extern thread_local std::string g_err;

}  // namespace vmg
