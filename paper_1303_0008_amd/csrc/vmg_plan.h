// Plan object of the gfx950 multigrid library (host side).
#pragma once
#include <hip/hip_runtime.h>

#include <string>
#include <vector>

#include "../../include/vmg.h"
#include "vmg_internal.h"

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

struct Plan {
    std::vector<GridState> grids;
    vmg_params params;
    Coef coef;
    hipStream_t stream = nullptr;
    hipStream_t own_stream = nullptr;      // created when the caller passes stream 0
    SmoothCfg cfg;
    int nu1 = 2, nu2 = 2, ncoarse = 40;
    bool periodic = true;
    bool mixed = false;
    bool has_source = false;
    bool solved = false;
    double* partials = nullptr;
    NormOut* host_norm = nullptr;          // pinned
    hipGraphExec_t graph[2];
    bool graph_ok[2] = {false, false};
    int64_t cell_updates = 0, finest_sweeps = 0;
    int64_t cycle_updates = 0, cycle_finest = 0;
    std::vector<void*> allocs;
};

vmg_status fail(vmg_status st, const std::string& msg);
CoefF make_coef_f(const Coef& c, double h);
vmg_status alloc_mixed(Plan* P);
hipError_t enqueue_outer(Plan* P);          // one mixed-precision outer iteration (+ norms to host)
hipError_t mixed_initial_pass(Plan* P);     // cast pass of the initial guess (+ norms to host)
hipError_t mixed_prepare(Plan* P);          // per-solve set-up of the FP32 ghost shells
hipError_t smooth_corr_level(Plan* P, GridState& G, int l);
extern thread_local std::string g_err;

}  // namespace vmg
