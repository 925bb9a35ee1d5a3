// Internal declarations of the gfx950 multigrid library (kernels <-> driver).
#pragma once
#include <hip/hip_runtime.h>
#include <cstdint>

namespace vmg {

// cells per work item of the batched (Dirichlet) passes: items are (grid, first
// cell) pairs over ITEM_CELLS consecutive cells of one grid
constexpr int ITEM_CELLS = 256;

// One level of one grid as the kernels see it.  Periodic levels are stored
// unpadded (n0*n1*n2, x fastest) and wrap their indices; Dirichlet levels are
// stored with a one-cell shell ((n0+2)*(n1+2)*(n2+2)) that holds the ghosts.
struct Geom {
    int n0, n1, n2;
    int dir;          // 1: Dirichlet (padded), 0: periodic
    int64_t sy, sz;   // element strides of y and z (x stride is 1)
    int64_t off0;     // element offset of interior cell (0,0,0)
    int64_t ncell;    // n0*n1*n2
    int64_t nstore;   // elements of storage
    double h;
    int64_t base;     // element offset where this grid's storage starts (pooled batches)
};

// Coefficients of the discrete operator (Sec. III.A/B with w = 1/3):
//   q = alpha*Sigma0 + kappa*delta, D = 1 + c8*q, Q = 2q/(1+sqrt D) or vertex.
struct Coef {
    double alpha, kappa;
    double c8;        // 8*alpha/3
    double vertex;    // -3/(4 alpha) (unused when alpha == 0: then D == 1)
    int sqrt_form;    // |alpha| >= 1e-2: the root is taken as (sqrt D - 1) 3/(4 alpha)
};

// FP32 coefficients of the inner (correction) operator of the mixed path.
struct CoefF {
    float alpha;
    float c8;        // 8*alpha/3
    float a34;       // 3/(4 alpha) (unused when alpha == 0)
    float a_ih4;     // alpha / h^4
    float h2;        // h^2
};

// Reduction slots written per block and summed by k_finalize.
enum { R_D2 = 0, R_D1, R_Q, R_F, R_PHI, R_GUARD, R_NONFIN, R_NSLOT };

// Device-resident per-level scalars.
struct LevelScalars {
    double cbar;      // compatibility constant in use (periodic), 0 otherwise
    double pad[7];
};

// Host-visible result of a norm pass.
struct NormOut {
    double rms;       // sqrt(mean d^2) with the updated cbar
    double cbar;      // updated cbar
    double mean_phi;
    double n_guard;
    double n_nonfinite;
    double sum_q;
    double tau_rms;   // RMS of tau^h on the next coarser level (mean-free on periodic grids)
    double pad;
};

// Fused red-black sweep tile configuration.
constexpr int TX = 64;

struct SmoothCfg {
    int ty;      // 4, 8, 12 or 16
    int zc;      // z planes per block
    int pipe = 1;   // 0: black one plane behind red, two barriers per plane step;
                    // 1: black two planes behind, one barrier (four-plane rings);
                    // PIPE_BRICK: no z march, BB_SIDE^3 bricks (ty, zc unused): up
                    // to two sweeps per launch on periodic levels below the finest,
                    // one on any level of a Dirichlet batch
};
constexpr int PIPE_BRICK = 2;
constexpr int BB_SIDE = 8;   // brick side of PIPE_BRICK

// Blocks a tiled pass should at least launch: four per compute unit.
constexpr int64_t MIN_TILED_BLOCKS = 1024;

// z planes per block of a tiled pass over n2 planes with xy_tiles tiles per
// plane: zc0, halved (down to 2, so restriction keeps its z pairs) while the
// launch would have fewer than MIN_TILED_BLOCKS blocks.  Coarse levels then
// spread over the chip instead of running long serial z-marches on a few CUs.
inline int level_zc(int64_t xy_tiles, int n2, int zc0 = 16) {
    int zc = zc0;
    while (zc > 2 && xy_tiles * ((n2 + zc - 1) / zc) < MIN_TILED_BLOCKS) zc >>= 1;
    return zc;
}

// Fused-sweep schedule of one level: the plan's (tuned) schedule, with the
// z chunk shortened and then the tile height lowered to 4 on small grids.
inline SmoothCfg level_cfg(int n0, int n1, int n2, SmoothCfg c) {
    const int64_t tx = (n0 + 63) / 64;
    auto blocks = [&](int ty, int zc) { return tx * ((n1 + ty - 1) / ty) * ((n2 + zc - 1) / zc); };
    c.zc = level_zc(tx * ((n1 + c.ty - 1) / c.ty), n2, c.zc);
    if (blocks(c.ty, c.zc) < MIN_TILED_BLOCKS && c.ty > 4) {
        c.ty = 4;
        c.zc = level_zc(tx * ((n1 + 3) / 4), n2, c.zc);
    }
    return c;
}

// ---- coarse tail (kernels_tail.hip) ----------------------------------------
// Periodic levels with at most TAIL_CELLS cells, down to the coarsest, in one
// single-workgroup launch (all arrays in LDS).
constexpr int TAIL_CELLS = 512;
constexpr int TAIL_LEVELS = 6;
struct TailArgs {
    int nlev;                           // levels in the tail; [0] is its top level
    int n[TAIL_LEVELS][3];
    double h[TAIL_LEVELS];
    const double* delta[TAIL_LEVELS];   // density of each level (device, x fastest)
    double* phi;                        // top-level state (in/out)
    const double* f;                    // top-level FAS rhs (may be null: zero)
    LevelScalars* sc;                   // top-level cbar (in/out)
    Coef c;
    int nu1, nu2, ncoarse;
};
hipError_t launch_tail(const TailArgs& a, hipStream_t s);
// the same for the mixed path's FP32 correction problem
struct TailCorrArgs {
    int nlev;
    int n[TAIL_LEVELS][3];
    double h[TAIL_LEVELS];
    const double* delta[TAIL_LEVELS];   // density of each level (t0 below the top level)
    float* e;                           // top-level correction (in/out)
    const float* r;                     // top-level rhs of the correction problem
    const float* pt;                    // top-level base state phi~
    const float* t0;                    // top-level +-sqrt|D0|
    LevelScalars* sc;                   // top-level inner cbar (in/out)
    Coef c64;                           // FP64 coefficients (alpha, c8, kappa)
    int nu1, nu2, ncoarse;
};
hipError_t launch_tail_corr(const TailCorrArgs& a, hipStream_t s);

// ---- launchers (kernels.hip) --------------------------------------------
// Coarse correction prolonged inside a sweep: the sweep starts from
// u^h + P(uc - oc) (cell-centred trilinear) instead of u^h.
template <typename T>
struct ProlongInT {
    Geom gc;
    const T* uc;
    const T* oc;
};
using ProlongIn = ProlongInT<double>;
using ProlongInF = ProlongInT<float>;
// The folded prolongation needs a periodic grid twice the coarse one per axis
// and an even z chunk (the coarse planes are staged on odd steps).
inline bool can_fold_prolong(const Geom& g, const Geom& gc, int zc) {
    return !g.dir && !gc.dir && (zc & 1) == 0 && g.n0 == 2 * gc.n0 && g.n1 == 2 * gc.n1 && g.n2 == 2 * gc.n2;
}
// Where folding pays (measured on 128^3-512^3 solves): a z chunk of at least 8
// planes amortises the block's start-up (four coarse planes staged, three ring
// planes corrected), and on levels of at most 64^3 cells the saved launch
// outweighs it.  A 128^3 level swept in chunks of 4 loses.
inline bool fold_prolong_pays(const Geom& g, int zc) { return zc >= 8 || g.ncell <= (int64_t)1 << 18; }
// nsweeps: sweeps of this launch (2 only with the brick schedule)
hipError_t launch_smooth(const Geom& g, const Coef& c, const double* pin, double* pout,
                         const double* delta, const double* f, const LevelScalars* sc,
                         SmoothCfg cfg, hipStream_t s, const ProlongIn* pro = nullptr, int nsweeps = 1);
hipError_t launch_residual_restrict(const Geom& gf, const Geom& gc, const Coef& c,
                                    const double* phi, const double* delta, const double* f,
                                    const LevelScalars* sc, double* phic, double* phiold_c,
                                    double* rd_c, double* partials, int* nblocks_out, hipStream_t s);
hipError_t launch_residual_norm(const Geom& g, const Coef& c, const double* phi,
                                const double* delta, const double* f, const LevelScalars* sc,
                                double* d_out, double* partials, int* nblocks_out, hipStream_t s);
hipError_t launch_fas_rhs(const Geom& g, const Coef& c, const double* phi, const double* delta,
                          const double* rd, double* f, double* partials, int* nblocks_out,
                          hipStream_t s,
                          const double* f_fine = nullptr, const Geom* gfine = nullptr);
// mode 0: residual pass (updates cbar from sum Q + sum f, corrects the lagged sums, writes NormOut)
// mode 1: FAS rhs pass (cbar = mean f + mean Q; with `out`, also out->tau_rms)
// mode 2: as mode 0, and also sets inner->cbar = -mean(d) (mean of the inner right-hand side)
hipError_t launch_finalize(const double* partials, int nblocks, int64_t ncell, int periodic,
                           int mode, LevelScalars* sc, NormOut* out, hipStream_t s,
                           LevelScalars* inner = nullptr);
// One reduction of a pass's block partials (the arguments of launch_finalize).
struct FinJob {
    const double* partials;
    int nblocks, periodic, mode;
    int64_t ncell;
    LevelScalars* sc;
    NormOut* out;
    LevelScalars* inner;
};
struct FinJobs {
    FinJob j[2];
};
// Two independent reductions in one launch (one block each).
hipError_t launch_finalize_pair(const FinJob& a, const FinJob& b, hipStream_t s);
hipError_t launch_prolong(const Geom& gf, const Geom& gc, double* phif, const double* phic,
                          const double* phiold_c, hipStream_t s);
hipError_t launch_coarse_solve(const Geom& g, const Coef& c, double* phi, const double* delta,
                               const double* f, LevelScalars* sc, int sweeps, hipStream_t s);
hipError_t launch_restrict_plain(const Geom& gf, const Geom& gc, const double* uf, double* uc,
                                 hipStream_t s);
hipError_t launch_copy_in(const Geom& g, const double* src, double* dst, hipStream_t s);
hipError_t launch_copy_out(const Geom& g, const double* src, double* dst, hipStream_t s);
hipError_t launch_ghost_in(const Geom& g, const double* ghost, double* dst, hipStream_t s);
hipError_t launch_restrict_ghosts(const Geom& gf, const Geom& gc, const double* uf, double* uc,
                                  hipStream_t s);
hipError_t launch_gauge(const Geom& g, double* phi, const NormOut* no, hipStream_t s);
hipError_t launch_fill(double* p, int64_t n, double v, hipStream_t s);
hipError_t launch_check_finite(const double* p, int64_t n, double* partials, int* nblocks_out,
                               hipStream_t s);
hipError_t launch_ghost_fill(const double* parent, int np0, int np1, int np2, double H,
                             int n0, int n1, int n2, double h, int o0, int o1, int o2,
                             double* ghost, hipStream_t s);
// Psi = phi_N + phi/2 (psi may be null) and g = -grad Psi (gx, gy, gz blocks of N), periodic
hipError_t launch_total_force(int n0, int n1, int n2, double h, const double* phin, const double* phi, double* psi,
                              double* g, hipStream_t s);
int64_t total_force_blocks(int n0, int n1, int n2);
hipError_t launch_interior_fill(const double* parent, int np0, int np1, int np2, double H, int n0, int n1, int n2,
                                double h, int o0, int o1, int o2, double* phi, hipStream_t s);
// Particles (np x 3, box units) -> delta on a periodic n0 x n1 x n2 grid;
// scheme 1 cloud in cell, 2 triangular-shaped cloud (kernels_assign.hip).
// work: mass_assign_workspace(np, n0, n1, n2) bytes, 256-byte aligned.
int64_t mass_assign_bricks(int n0, int n1, int n2);
int64_t mass_assign_workspace(int64_t np, int n0, int n1, int n2);
// The allocation-free variant's workspace: a static device array of
// NOALLOC_SCRATCH_BYTES per GPU; noalloc_scratch() gives the current device's
// address (looked up with hipGetSymbolAddress on a device's first call).
constexpr int64_t NOALLOC_SCRATCH_BYTES = int64_t(64) << 20;
constexpr int NOALLOC_MAX_DEVICES = 64;
hipError_t noalloc_scratch(void** ptr);
// periodic: the whole box (h, corner unused); else a region of cells of size h
// whose cell (0,0,0) corner is at corner[3].  delta = mass / mean_count - 1.
hipError_t launch_mass_assign(const double* pos, int64_t np, int n0, int n1, int n2, int scheme, bool periodic,
                              double h, const double* corner, double mean_count, void* work, double* delta,
                              hipStream_t s);

// ---- mixed path (kernels_mixed.hip) ---------------------------------------
// zero_in: the input correction is identically zero (first sweep of an inner
// cycle); ein is then not read.
hipError_t launch_smooth_corr(const Geom& g, const CoefF& c, const float* ein, float* eout,
                              const float* pt, const float* t0, const float* r, const LevelScalars* sc,
                              SmoothCfg cfg, hipStream_t s, bool zero_in = false,
                              const ProlongInF* pro = nullptr, int nsweeps = 1);
// ptc (may be null): receives the restricted base state phi~ of the coarse level
hipError_t launch_rr_corr(const Geom& gf, const Geom& gc, const CoefF& c, const float* e, const float* pt,
                          const float* t0, const float* r, const LevelScalars* sc, float* ec, float* eold_c,
                          float* rd_c, float* ptc, double* partials, int* nblocks_out, hipStream_t s);
// fresh_base: also computes and writes the level's t0 from phi~ and delta (FP64
// discriminant); otherwise reads the t0 a previous call wrote (same base state)
hipError_t launch_fas_corr(const Geom& g, const CoefF& c, const Coef& c64, const double* delta, const float* e,
                           const float* pt, float* t0, const float* rd, float* r, double* partials,
                           int* nblocks_out, hipStream_t s, bool fresh_base = true);
hipError_t launch_prolong_corr(const Geom& gf, const Geom& gc, float* ef, const float* ec, const float* eold_c,
                               hipStream_t s);
hipError_t launch_coarse_corr(const Geom& g, const CoefF& c, float* e, const float* pt, const float* t0,
                              const float* r, int sweeps, hipStream_t s);
hipError_t launch_cast(const Geom& g, const Coef& c, const double* phi, const double* delta, const double* f,
                       const LevelScalars* sc, float* pt, float* t0, float* r, double* partials,
                       int* nblocks_out, hipStream_t s);
// phi_out = phi + e (e may be null: then phi_out is not written), FP64 residual of it,
// norm partials and the FP32 inner inputs (pt, t0, r)
hipError_t launch_cast_update(const Geom& g, const Coef& c, const double* phi, const float* e, double* phi_out,
                              const double* delta, const double* f, const LevelScalars* sc, float* pt, float* t0,
                              float* r, double* partials, int* nblocks_out, hipStream_t s);
hipError_t launch_base_restrict(const Geom& gf, const Geom& gc, const float* pf, float* pc, hipStream_t s);
hipError_t launch_base_t0(const Geom& g, const Coef& c, const float* pt, const double* delta, float* t0,
                          hipStream_t s);
hipError_t launch_update(const Geom& g, double* phi, const float* e, hipStream_t s);
hipError_t launch_fill_f(float* p, int64_t n, float v, hipStream_t s);
hipError_t launch_cast_all(const double* src, float* dst, int64_t n, hipStream_t s);

// ---- batched Dirichlet launchers (one launch per level for every grid) ------
struct SmoothArgs;
// one sweep of every grid of a batched level; gref (brick schedule only, levels
// below the finest): refresh pout's ghost shell against this reference as well
hipError_t launch_smooth_batch_args(const Coef& c, const double* pin, double* pout, const double* delta,
                                    const double* f, SmoothCfg cfg, const Geom* geoms, const int4* items,
                                    int nitems, int max_blocks, hipStream_t s, const double* gref = nullptr);
// items: the coarse level's cells; also sets the coarse ghost shell of phic to phiold_c's
hipError_t launch_rr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, const Coef& c,
                           const double* phi, const double* delta, const double* f, double* phic,
                           double* phiold_c, double* rd_c, hipStream_t s);
hipError_t launch_fas_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                            const double* delta, const double* rd, double* f, hipStream_t s);
// items: the coarse level's cells (each thread updates the 8 children of one)
hipError_t launch_prolong_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, double* phif,
                                const double* phic, const double* oldc, hipStream_t s);
// tau^h of every grid on level 1 (items: level-1 cells; first: each grid's block
// range in them) into out[k].tau_rms; phi, delta, rd are the level-1 pools after
// launch_rr_batch and the ghost refresh, f_fine the finest level's f (or null)
hipError_t launch_tau_batch(const Geom* gs, const Geom* gfs, const int2* items, int nitems, const Coef& c,
                            const double* phi, const double* delta, const double* rd, const double* f_fine,
                            double* partials, const int* first, int ngrids, NormOut* out, hipStream_t s);
hipError_t launch_norm_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                             const double* delta, const double* f, double* partials, const int* first, int ngrids,
                             NormOut* out, hipStream_t s);
hipError_t launch_finalize_batch(const double* partials, const int* first, const Geom* gs, int ngrids,
                                 NormOut* out, hipStream_t s);
hipError_t launch_coarse_batch(const Geom* gs, int ngrids, const Coef& c, double* phi0, double* phi1,
                               const double* delta, const double* f, int sweeps, const double* old,
                               hipStream_t s);
hipError_t launch_ghost_refresh_batch(const Geom* gs, const int2* items, int nitems, double* u, const double* ref,
                                      hipStream_t s);
hipError_t launch_ghost_refresh_batch_f(const Geom* gs, const int2* items, int nitems, float* u, const float* ref,
                                        hipStream_t s);
hipError_t launch_copy_in_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                const double* src, double* dst0, double* dst1, hipStream_t s);
hipError_t launch_copy_out_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                 const double* src, double* dst, hipStream_t s);
hipError_t launch_ghost_in_batch(const Geom* gs, const int64_t* goff, const int2* items, int nitems,
                                 const double* ghost, double* dst0, double* dst1, hipStream_t s);
hipError_t launch_restrict_plain_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                       const double* uf, double* uc, hipStream_t s);
hipError_t launch_restrict_ghosts_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                        const double* uf, double* uc0, double* uc1, double* uc2, hipStream_t s);
hipError_t launch_check_finite_batch(const Geom* gs, const int64_t* uoff, const int2* items, int nitems,
                                     const double* src, double* partials, hipStream_t s);
hipError_t launch_smooth_corr_batch(const CoefF& c, const float* ein, float* eout, const float* pt, const float* t0,
                                    const float* r, SmoothCfg cfg, const Geom* geoms, const int4* items, int nitems,
                                    int max_blocks, hipStream_t s, const float* gref = nullptr);
// items: the coarse level's cells; also sets the coarse ghost shell of ec to eold_c's
hipError_t launch_rr_corr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, const CoefF& c,
                                const float* e, const float* pt, const float* t0, const float* r, float* ec,
                                float* eold_c, float* rd_c, hipStream_t s);
hipError_t launch_fas_corr_batch(const Geom* gs, const int2* items, int nitems, const CoefF& c, const float* e,
                                 const float* pt, const float* t0, const float* rd, float* r, hipStream_t s);
// items: the coarse level's cells
hipError_t launch_prolong_corr_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems, float* ef,
                                     const float* ec, const float* eold_c, hipStream_t s);
hipError_t launch_coarse_corr_batch(const Geom* gs, int ngrids, const CoefF& c, float* e0, float* e1,
                                    const float* pt, const float* t0, const float* r, int sweeps, const float* old,
                                    hipStream_t s);
hipError_t launch_cast_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const double* phi,
                             const double* delta, const double* f, float* pt, float* t0, float* r,
                             double* partials, hipStream_t s);
hipError_t launch_base_restrict_batch(const Geom* gfs, const Geom* gcs, const int2* items, int nitems,
                                      const float* pf, float* pc, hipStream_t s);
hipError_t launch_base_t0_batch(const Geom* gs, const int2* items, int nitems, const Coef& c, const float* pt,
                                const double* delta, float* t0, hipStream_t s);
hipError_t launch_update_batch(const Geom* gs, const int2* items, int nitems, double* phi, const float* e,
                               hipStream_t s);

int64_t ghost_count(int n0, int n1, int n2);
int partial_blocks_for(int64_t ncell);   // upper bound of blocks used by grid-stride reduction kernels
int resid_blocks(const Geom& g);         // blocks of the tiled residual kernel on level g

}  // namespace vmg
