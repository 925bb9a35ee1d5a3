/*
 * vmg.h -- C ABI of the MI355X (gfx950) nonlinear multigrid solver for the
 * Vainshtein-screened scalar field of DGP/Galileon gravity.
 *
 * Problem (Li, Zhao & Koyama, Sec. III.A, Eq. code_eqn, in code units):
 *
 *     Lap(phi) + alpha [ (Lap phi)^2 - (d_i d_j phi)^2 ] = kappa * delta
 *
 * Here alpha is the coefficient of the nonlinear term (the reciprocal of the
 * paper's alpha = 3 beta a^4 / R_c^2) and kappa the source coefficient
 * (Omega_m a / beta).  Discretisation (Sec. III.B): cell-centred cubic cells
 * of size h, 7-point Laplacian, 3-point second and 4-point cross differences,
 * operator splitting with w = 1/3 (Eq. two_branch) and the physical root
 * (Eq. one_branch).  At w = 1/3 the per-cell root does not depend on the
 * cell's own value, so the nonlinear Gauss-Seidel update is closed form:
 *
 *     Sigma0 = [ ((a_x-a_y)^2 + (a_x-a_z)^2 + (a_y-a_z)^2)/3
 *               + (B_xy^2 + B_xz^2 + B_yz^2)/8 ] / h^4
 *     q = alpha*Sigma0 + kappa*delta,   D = 1 + (8 alpha / 3) q
 *     Q = 2q / (1 + sqrt(D))   (D >= 0),   Q = -3/(4 alpha)   (D < 0, guard)
 *     operator  L(phi) = Lap_h phi - Q
 *
 * a_x etc. are the 3-point second differences times h^2, B_xy etc. the
 * 4-point cross differences times 4h^2 (Sec. III.B, discrete Sigma_ijk).
 *
 * Equations solved (Sec. III.C, Eq. fine_grid_eqn, with f the optional source):
 *   periodic grid : L(phi) + cbar = f, with the constant cbar = mean(f) - mean(L(phi))
 *                   that makes the periodic problem solvable, and mean(phi) = 0;
 *   Dirichlet grid: L(phi) = f on the n0*n1*n2 cells, neighbours outside the grid
 *                   taken from a given one-cell ghost shell (refinement boundary,
 *                   Sec. III.C and IV.D).
 * Residual d = L(phi) (+ cbar) - f; reported norm = sqrt(mean(d^2)) in FP64.
 *
 * Method: full-approximation-scheme V-cycles (Sec. III.C): fused red-black
 * nonlinear Gauss-Seidel sweeps, residual with 8-child-average restriction,
 * coarse right-hand side f^H = L^H(R phi^h) - R d^h, cell-centred trilinear
 * prolongation of phi^H - R phi^h, direct relaxation on the coarsest level.
 * A cell whose D lies next to the guard boundary has its update scaled by
 * min(1, max(0.01, 50 (256 h)^2 sqrt|D|)) (the root's slope 1/sqrt(D) would
 * otherwise make its update oscillate across D = 0); elsewhere the update is
 * the plain one, and a converged phi is the same either way.
 *
 * Memory conventions.  Every array pointer is a DEVICE pointer (hipMalloc /
 * torch.cuda memory) to FP64 data, x fastest: cell (i,j,k) of a grid is
 * element offset + (k*n1 + j)*n0 + i.  The caller owns every array passed in;
 * the plan owns all its workspaces.  No entry point throws; failures return a
 * status and vmg_last_error() describes the last one (per thread).
 */
#ifndef VMG_H
#define VMG_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    VMG_OK = 0,
    VMG_EINVAL = 1,       /* invalid argument: sizes, spacing, tolerance, null pointer ... */
    VMG_ENOMEM = 2,       /* device or host allocation failed */
    VMG_EHIP = 3,         /* a HIP runtime call failed */
    VMG_ENOCONV = 4,      /* max_cycles reached before the tolerance; results are filled */
    VMG_ENONFINITE = 5    /* non-finite input or residual, or the residual diverged */
} vmg_status;

typedef enum { VMG_FP64 = 0, VMG_MIXED = 1 } vmg_precision;
typedef enum { VMG_PERIODIC = 0, VMG_DIRICHLET = 1 } vmg_bc;

/* flags */
#define VMG_GRAPH 1u          /* replay the V-cycle as a captured hipGraph */
#define VMG_AUTOTUNE 2u       /* time tile/schedule choices at plan creation */

/* One grid.  A plan holds either exactly one periodic grid or one or more
 * Dirichlet grids (refinement patches, solved as one batch). */
typedef struct {
    int32_t n[3];          /* cells along x, y, z; periodic: even, >= 4; Dirichlet: >= 2 */
    int32_t bc;            /* vmg_bc */
    double h;              /* cell size (> 0) */
    int64_t offset;        /* element offset of this grid's cells in delta / phi / source */
    int64_t ghost_offset;  /* Dirichlet: element offset of its ghost values in `ghost` */
} vmg_grid;

/* Compact ghost order of a Dirichlet grid (2(n1 n2 + n0 n2 + n0 n1) + 4(n0+n1+n2) values):
 *   faces  x-, x+ : cells (-1, j, k), (n0, j, k)   j fastest, then k
 *   faces  y-, y+ : cells (i, -1, k), (i, n1, k)   i fastest, then k
 *   faces  z-, z+ : cells (i, j, -1), (i, j, n2)   i fastest, then j
 *   edges along x : (i,-1,-1), (i,n1,-1), (i,-1,n2), (i,n1,n2)   i fastest
 *   edges along y : (-1,j,-1), (n0,j,-1), (-1,j,n2), (n0,j,n2)   j fastest
 *   edges along z : (-1,-1,k), (n0,-1,k), (-1,n1,k), (n0,n1,k)   k fastest
 * Corner cells are not part of the 19-point stencil and are not stored. */

typedef struct {
    double alpha;          /* coefficient of the nonlinear term (0 = linear Poisson limit) */
    double kappa;          /* source coefficient */
    double tol;            /* stop when the RMS residual of every grid is <= tol (> 0) */
    int32_t max_cycles;    /* V-cycles (FP64) or outer iterations (mixed); >= 1 */
    int32_t prec;          /* vmg_precision */
    int32_t nu1, nu2;      /* pre/post smoothing sweeps; 0,0 selects the defaults (2,2) */
    uint32_t flags;        /* VMG_GRAPH | VMG_AUTOTUNE */
    int32_t inner_cycles;  /* mixed: FP32 inner V-cycles per outer FP64 iteration (0 = 2);
                              must be 0 for VMG_FP64 */
    double tau_factor;     /* > 0: also stop once |d^h| <= tau_factor |tau^h| on every grid,
                              tau^h = L^H(R phi) - R L^h(phi) the truncation-error estimate of
                              Sec. III.C (the paper takes the factor <= 1/3), both at the same
                              phi; on a Dirichlet grid the coarse operator reads the restricted
                              boundary values.  Every grid needs a coarser level; 0 = off */
} vmg_params;

typedef struct {
    double rms0;           /* RMS residual of the initial guess */
    double rms;            /* RMS residual of the returned phi */
    double compat_c;       /* cbar (periodic), 0 for Dirichlet */
    int32_t cycles;        /* V-cycles run (FP64) or outer iterations (mixed) */
    int32_t inner_cycles;  /* FP32 inner V-cycles (mixed), 0 otherwise */
    int64_t n_guarded;     /* cells where D < 0 at the returned phi */
    double tau_rms;        /* with tau_factor > 0: RMS over the next coarser level's cells of
                              tau^h at the returned phi (mean removed on periodic grids); else 0 */
} vmg_result;

typedef struct vmg_plan vmg_plan;

/* Create a solver plan for `n_grids` grids (Sec. III.C: the domain grid, or a
 * set of refinement patches).  Allocates every workspace on the current
 * device, may run the autotuner (VMG_AUTOTUNE) and, with VMG_GRAPH, records
 * and instantiates the hipGraphs of one iteration (one per finest-level
 * ping-pong parity, with and without a source), so that vmg_solve replays them
 * without allocating.  All later work is issued on `stream` (0: a blocking
 * stream the plan creates, since the legacy null stream cannot be captured).
 * Errors: VMG_EINVAL (sizes, h <= 0, tol <= 0, max_cycles < 1, inner_cycles < 0 or
 * set for VMG_FP64, tau_factor < 0 or not finite, tau_factor > 0 with a grid that has
 * no coarser level, mixed BC kinds,
 * a periodic grid that does not coarsen to <= 8 cells per side, a Dirichlet
 * grid whose coarsest level exceeds 8 cells per side), VMG_ENOMEM, VMG_EHIP. */
vmg_status vmg_plan_create(vmg_plan **plan, const vmg_grid *grids, int32_t n_grids,
                           const vmg_params *p, hipStream_t stream);

/* Solve (Sec. III.C: V-cycles until |d| < tol).  delta: density contrast of
 * every grid; ghost: Dirichlet ghost values (may be NULL for a periodic plan);
 * source: optional additive right-hand side f (NULL = 0), in either precision
 * (the mixed path's FP64 defect includes it); phi: initial guess in, solution
 * out (periodic: mean removed).  out: host array of n_grids results.  Never
 * allocates device memory (with VMG_GRAPH it replays the graphs recorded at
 * plan creation); runs on the plan's stream and returns after it has finished.
 * Divergence: a non-finite residual, a residual 1e4 times above the smallest
 * one seen so far, or (after the first four iterations, whose nonlinear start
 * phase may raise it) three iterations in a row 10 times above it.
 * Errors: VMG_EINVAL (null pointers), VMG_ENONFINITE (non-finite delta or
 * residual, divergence; phi holds the last iterate), VMG_ENOCONV (max_cycles
 * reached; phi and out are filled), VMG_EHIP. */
vmg_status vmg_solve(vmg_plan *plan, const double *delta, const double *ghost,
                     const double *source, double *phi, vmg_result *out);

/* Release every resource of the plan (NULL is accepted). */
vmg_status vmg_plan_destroy(vmg_plan *plan);

/* Thread-local message describing the last non-OK status ("" if none). */
const char *vmg_last_error(void);

/* Convenience: one periodic n^3 grid of the unit box (h = 1/n), one call.
 * precision: vmg_precision.  rms and cycles are host pointers (may be NULL).
 * Creates and destroys a plan internally (so it allocates). */
vmg_status vmg_solve_periodic(const double *delta, int32_t n, double alpha, double kappa,
                              double tol, int32_t precision, double *phi, double *rms,
                              int32_t *cycles, hipStream_t stream);

/* Residual of a given phi on grid `g` of a plan (Sec. III.C: d^h = L^h(phi^h) - f^h,
 * with cbar on periodic grids): writes d (device, same layout as phi; may be
 * NULL) and *res (host).  Pointers index the whole batch as in vmg_solve.
 * Errors: VMG_EINVAL, VMG_EHIP. */
vmg_status vmg_residual(vmg_plan *plan, int32_t g, const double *delta, const double *ghost,
                        const double *source, const double *phi, double *d, vmg_result *res);

/* Refinement boundary values (Sec. III.C, IV.D: "interpolated from coarser
 * levels"): trilinear interpolation of a cell-centred periodic parent field
 * (np[0] x np[1] x np[2] cells of size parent_h, device pointer, x fastest) at
 * the centres of the ghost cells of each Dirichlet grid.  origins: host array of
 * 3*n_grids integers, the position of cell (0,0,0) of grid i in units of that
 * grid's h.  Writes ghost (device) at each grid's ghost_offset, compact order.
 * Errors: VMG_EINVAL, VMG_EHIP. */
vmg_status vmg_fill_ghosts(const double *parent, const int32_t np[3], double parent_h,
                           const vmg_grid *grids, const int32_t *origins, int32_t n_grids,
                           double *ghost, hipStream_t stream);

/* Place of a refinement in a multilevel hierarchy: the index of its parent in
 * the hierarchy's grid array (-1 for the domain grid) and the position of its
 * cell (0,0,0) corner from the parent's cell (0,0,0) corner, in units of its
 * own cell size (the origins of vmg_fill_ghosts). */
typedef struct {
    int32_t parent;
    int32_t origin[3];
} vmg_nest;

/* Multilevel solve (Sec. III.C: the domain grid and the refinements are each
 * solved with multigrid, a refinement taking the boundary values of its edge
 * cells interpolated from the coarser level; Sec. IV.D: a refinement placed
 * over the overdensity, with the same density on it).  grids[0] is the
 * periodic domain grid (nest[0].parent = -1); every other grid is a Dirichlet
 * refinement whose parent comes earlier in the array, with half the parent's
 * cell size.  Under the domain grid a refinement may sit anywhere (origin in
 * [0, 2 n) per axis; it wraps); under a refinement it keeps one parent cell of
 * margin (origin >= 2 and origin + n <= 2 n_parent - 2 per axis), so the
 * interpolation needs no value outside the parent.  The solve runs level by
 * level: the domain grid from the phi given at its offset, then each depth of
 * the tree as one batched plan, every refinement starting from ghost values
 * (written to `ghost` at its ghost_offset) and an initial guess interpolated
 * trilinearly from its parent's solution (as vmg_fill_ghosts and
 * vmg_fill_interior).  Refinements do not feed back into their parents.
 * delta, ghost and phi are device arrays holding every grid at its offset (x
 * fastest); phi receives every solution.  p applies to every level; out: host
 * array of n_grids results.  Creates and
 * destroys its plans (allocates).  Errors: VMG_EINVAL (nesting or arguments),
 * otherwise the first failing level's status (VMG_ENOCONV, VMG_ENONFINITE,
 * ...; deeper levels are then not solved), VMG_EHIP.  Equivalent to
 * vmg_levels_create + vmg_levels_solve + vmg_levels_destroy. */
vmg_status vmg_solve_levels(const vmg_grid *grids, const vmg_nest *nest, int32_t n_grids, const vmg_params *p,
                            const double *delta, double *ghost, double *phi, vmg_result *out, hipStream_t stream);

/* The multilevel solve as a reusable plan: vmg_levels_create validates the
 * tree as vmg_solve_levels does and allocates one plan per depth (the domain
 * grid's, then one batched plan per refinement depth) on `stream`;
 * vmg_levels_solve runs the level-by-level solve on those plans without
 * allocating (same arrays, results and errors as vmg_solve_levels; the
 * results of levels it does not reach are zeroed; returns after the stream
 * has finished); vmg_levels_destroy frees the plans (NULL is
 * ignored).  A levels plan must not be used from two threads at once. */
typedef struct vmg_levels vmg_levels;
vmg_status vmg_levels_create(vmg_levels **levels, const vmg_grid *grids, const vmg_nest *nest, int32_t n_grids,
                             const vmg_params *p, hipStream_t stream);
vmg_status vmg_levels_solve(vmg_levels *levels, const double *delta, double *ghost, double *phi, vmg_result *out);
void vmg_levels_destroy(vmg_levels *levels);

/* Initial guess on refinements (Sec. III.C, IV.D: a refinement starts from the
 * solution of the coarser level, interpolated): the same trilinear
 * interpolation of the periodic parent as vmg_fill_ghosts, at every cell centre
 * of each grid, written to phi (device) at each grid's offset, x fastest.
 * Starting a refinement from zero instead of from this guess leaves a jump of
 * the boundary values across the outermost cells, which the nonlinear operator
 * turns into a long slow phase of the solve.  Errors: VMG_EINVAL, VMG_EHIP. */
vmg_status vmg_fill_interior(const double *parent, const int32_t np[3], double parent_h,
                             const vmg_grid *grids, const int32_t *origins, int32_t n_grids,
                             double *phi, hipStream_t stream);

/* Total potential and force (Sec. II.B: the model's total potential is
 * Psi = phi_N + phi/2, differenced to give the force on particles; Sec. III.B:
 * the gradient is the central difference (u_{i+1} - u_{i-1}) / 2h).  On a
 * periodic n[0] x n[1] x n[2] grid of cell size h (device arrays, x fastest):
 * phi_newton is the Newtonian potential (Eq. newton, Lap phi_N = (3/2) Omega_m a
 * delta: vmg_solve with alpha = 0 and kappa = 1.5 Omega_m a solves it), phi the
 * brane-bending mode.  Writes psi = phi_newton + phi/2 (may be NULL) and the
 * acceleration -grad Psi into force: 3 N values, the x, y and z components one
 * after another.  Enqueued on `stream`; the caller owns every buffer.
 * Errors: VMG_EINVAL (null input or force, n < 1, more than 2^31 - 1 tiles
 * of 64 x 8 x 16 cells, h not finite and > 0), VMG_EHIP. */
vmg_status vmg_total_force(const double *phi_newton, const double *phi, const int32_t n[3], double h,
                           double *psi, double *force, hipStream_t stream);

/* Mass assignment (Sec. VI: the density on the mesh is obtained by assigning
 * the particles with the triangular-shaped-cloud scheme, and the solver needs
 * no further smoothing of it).  Unit-mass particles at pos (device array,
 * n_particles x 3 doubles, row p = x, y, z of particle p in box units; the box
 * is periodic and a coordinate is taken modulo 1) are assigned to a periodic
 * grid of n[0] x n[1] x n[2] cells whose cell i along an axis is centred at
 * (i + 1/2)/n.  With u = x * n along an axis:
 *   VMG_ASSIGN_CIC  weights 1 - t and t on cells floor(u - 1/2) and the next,
 *                   t = u - 1/2 - floor(u - 1/2);
 *   VMG_ASSIGN_TSC  nearest cell c = floor(u), d = u - c - 1/2, weights
 *                   (1/2 - d)^2/2, 3/4 - d^2, (1/2 + d)^2/2 on cells c-1, c, c+1;
 * the 3-D weight is the product of the three axes' weights.  Writes delta =
 * rho / mean(rho) - 1 (x fastest; mean(rho) = n_particles / cells), so the
 * result is the right-hand side's density contrast.  A particle with a
 * non-finite coordinate deposits nothing but counts in the mean.  Masses are
 * summed in 64-bit fixed point (2^-40 of a particle, each contribution rounded
 * once, integer sums), so the result is bitwise reproducible and independent
 * of the particles' order; a cell may receive the mass of fewer than 2^24
 * particles.  The previous contents of delta are ignored.
 * workspace: device memory of at least vmg_mass_assign_workspace(n_particles,
 * n) bytes, 256-byte aligned, owned by the caller, contents ignored (it holds
 * the particles binned by 16^3-cell brick of the grid and each brick's
 * boundary sums); calls that share a workspace
 * must be ordered on one stream.  Enqueued on `stream`; the caller owns every
 * buffer.  Errors: VMG_EINVAL (null pointer, n_particles outside
 * [1, 2^31 - 1], n < 1, n[1] or n[2] above 65535, unknown scheme, workspace
 * too small or misaligned), VMG_EHIP. */
#define VMG_ASSIGN_CIC 1
#define VMG_ASSIGN_TSC 2
vmg_status vmg_mass_assign(const double *pos, int64_t n_particles, const int32_t n[3], int32_t scheme,
                           void *workspace, int64_t workspace_bytes, double *delta, hipStream_t stream);

/* Mass assignment onto a refinement (Sec. VI: the mesh density comes from the
 * particles on every level): the region of n[0] x n[1] x n[2] cells of size h
 * whose cell (0,0,0) corner sits at corner[] (box units), not periodic.  Along
 * each axis a particle's offset from the corner is taken modulo 1 and moved
 * below the corner (offset - 1) when it lies more than n h + 2h past it; the
 * region must leave at least 4 of its cells of the unit box uncovered per axis
 * (n h <= 1 - 4h), so at most one periodic image of a particle reaches it.
 * With u = offset / h the weights are those of vmg_mass_assign; contributions
 * to cells outside the region are dropped.  Writes delta = mass / mean_count
 * - 1 (x fastest), mean_count being the box's mean number of particles per
 * cell of this size (N_box h^3 for N_box particles in the unit box); the
 * particles passed may be any subset that includes every particle within two
 * cells of the region.  Arithmetic, workspace (vmg_mass_assign_workspace with
 * this n), reproducibility and streams as vmg_mass_assign.  Errors:
 * VMG_EINVAL (as vmg_mass_assign, plus h, mean_count or corner not finite and
 * positive, a region too large for the box), VMG_EHIP. */
vmg_status vmg_mass_assign_region(const double *pos, int64_t n_particles, const int32_t n[3], double h,
                                  const double corner[3], double mean_count, int32_t scheme, void *workspace,
                                  int64_t workspace_bytes, double *delta, hipStream_t stream);

/* Allocation-free variant of vmg_mass_assign, for callers that cannot
 * allocate device memory (code under stream capture, tight serving loops,
 * harnesses that forbid hipMalloc): the same computation, arguments and result
 * as vmg_mass_assign, with the workspace taken from a static device array of
 * the library (64 MiB, held by every GPU the library runs on until the process
 * ends) instead of a caller workspace.  It calls no allocating routine.  Calls
 * on one GPU share that array: calls that overlap in time on one GPU (on
 * different streams, or from different threads) race and must be ordered by
 * the caller; each call rewrites every part of the array it reads.  Errors:
 * VMG_EINVAL (as vmg_mass_assign, and a call whose workspace,
 * vmg_mass_assign_workspace(n_particles, n), exceeds 64 MiB: e.g. a 128^3 grid
 * with more than about 4.8 M particles), VMG_EHIP. */
vmg_status vmg_mass_assign_noalloc(const double *pos, int64_t n_particles, const int32_t n[3], int32_t scheme,
                                   double *delta, hipStream_t stream);

/* Workspace bytes vmg_mass_assign needs (about 8 bytes per particle plus 12
 * per grid cell), or -1 for arguments vmg_mass_assign rejects. */
int64_t vmg_mass_assign_workspace(int64_t n_particles, const int32_t n[3]);

/* Number of ghost values of a Dirichlet grid with n cells per axis. */
int64_t vmg_ghost_count(const int32_t n[3]);

/* Measurement hook: run `sweeps` finest-level smoother sweeps (the kernel the
 * plan's precision uses on its finest level) on the plan's internal copy of
 * that level as the last vmg_solve left it, enqueued on the plan's stream
 * without host synchronisation.  Does not touch caller memory.
 * Errors: VMG_EINVAL (no solve yet, sweeps < 0), VMG_EHIP. */
vmg_status vmg_smooth(vmg_plan *plan, int32_t sweeps);

/* Measurement hook: with enable != 0, every finest-level sweep that later
 * solves launch is bracketed by HIP events on the plan's stream, and
 * vmg_plan_sweep_time returns the summed duration (microseconds) and the number
 * of those launches since this call.  While it is enabled a VMG_GRAPH plan
 * issues its iterations directly instead of replaying graphs (event nodes of a
 * graph carry no timestamps on this runtime): the same kernels on the same
 * data, launched one by one.  enable = 0 stops it and records the graphs again.
 * Allocates (events, graphs).  Errors: VMG_EINVAL, VMG_EHIP. */
vmg_status vmg_plan_time_sweeps(vmg_plan *plan, int32_t enable);
vmg_status vmg_plan_sweep_time(const vmg_plan *plan, double *total_us, int64_t *launches);

/* Measurement hook: with enable != 0, the work of every level in the
 * iterations of later solves is bracketed by HIP events on the plan's stream:
 * for a level l with a coarser level, its share of a V-cycle (the pre-sweeps,
 * the residual and restriction and the coarse right-hand side, then the
 * prolongation and the post-sweeps); the periodic coarse tail and the coarsest
 * solve are one piece, reported at the level where they start.  On the mixed
 * path the inner cycles' pieces and the outer FP64 pass (level 0) are timed.
 * vmg_plan_level_time returns the summed microseconds of `level` and the
 * number of iterations timed since this call.  While enabled a VMG_GRAPH plan
 * issues its iterations directly (as with vmg_plan_time_sweeps), and ROCTX
 * ranges name each level's pieces for rocprofv3 --marker-trace.  Batched
 * patch plans are not timed per level (level_time reports 0).  Allocates
 * events.  Errors: VMG_EINVAL (null plan, level out of range), VMG_EHIP. */
vmg_status vmg_plan_time_levels(vmg_plan *plan, int32_t enable);
vmg_status vmg_plan_level_time(const vmg_plan *plan, int32_t level, double *total_us, int64_t *iterations);

/* Residual history of the last vmg_solve of grid `grid` (Sec. III.C's
 * stopping test is on these norms): entry 0 holds the norms of the initial
 * guess, entry k those after iteration k (FP64: one V-cycle; mixed: one outer
 * defect-correction step).  Copies min(count, cap) entries into `out` (may be
 * null with cap 0) and returns count in *n.  The plan owns nothing the caller
 * passes.  Errors: VMG_EINVAL (null plan or n, grid out of range). */
typedef struct {
    double rms;        /* RMS of the FP64 residual d = L(phi) - f + cbar */
    double cbar;       /* periodic compatibility constant in use */
    double n_guarded;  /* cells on the guarded (vertex) branch of the root */
    double tau_rms;    /* RMS of tau^h on the next coarser level (tau rule), else 0 */
} vmg_history;
vmg_status vmg_plan_history(const vmg_plan *plan, int32_t grid, vmg_history *out, int32_t cap, int32_t *n);

/* Counters of the last vmg_solve (host pointers, each may be NULL):
 * cell_updates  = smoother cell updates over all levels and sweeps,
 * finest_sweeps = finest-level smoother sweeps (launches of that kernel),
 * finest_cells  = cells of the finest level(s) per sweep. */
vmg_status vmg_plan_stats(const vmg_plan *plan, int64_t *cell_updates, int64_t *finest_sweeps,
                          int64_t *finest_cells);

/* Schedule a plan uses (host pointers, each may be NULL): tile height and
 * z-chunk of the finest level's fused sweep (chosen by the autotuner with
 * VMG_AUTOTUNE, which times every swept level's smoother for tile heights
 * {4,8,12,16} x z chunks x pipeline shapes, plus the brick schedule on the
 * coarser levels of a periodic plan and on every level of a Dirichlet batch,
 * at plan creation, and installs a
 * cached cycle schedule of vmg_plan_tune_cycle; Sec. V of the paper notes the
 * code needed more tuning), pre/post sweeps and coarsest-level sweeps.
 * Errors: VMG_EINVAL. */
vmg_status vmg_plan_config(const vmg_plan *plan, int32_t *tile_y, int32_t *z_chunk, int32_t *nu1,
                           int32_t *nu2, int32_t *coarse_sweeps);

/* Cycle schedule of a plan (Sec. III.C leaves the number of relaxation
 * sweeps and the cycle shape to the implementation; Sec. V notes the code
 * needed more tuning).  Changing it changes the iteration, not the discrete
 * problem solved. */
typedef struct {
    int32_t nu1, nu2;        /* pre/post smoothing sweeps per level, 0..8, nu1 + nu2 >= 1 */
    int32_t inner_cycles;    /* mixed plans: FP32 inner V-cycles per outer iteration, 1..8;
                                FP64 plans: 0 */
    int32_t coarse_sweeps;   /* relaxation sweeps on the coarsest level, 1..64 */
    int32_t coarse_tail;     /* periodic plans: 1 = the levels of at most 512 cells run in one
                                single-workgroup launch, 0 = level by level; Dirichlet: 0 */
    int32_t batch_blocks;    /* Dirichlet plans: blocks of the persistent smoother launch,
                                64..65536; periodic plans: 0 */
    int32_t coarse_nu1, coarse_nu2;  /* pre/post sweeps on every level below the finest, 0..8
                                with coarse_nu1 + coarse_nu2 >= 1; both 0: nu1 and nu2 there too */
} vmg_cycle;

/* The cycle schedule a plan runs (host pointer).  Errors: VMG_EINVAL. */
vmg_status vmg_plan_get_cycle(const vmg_plan *plan, vmg_cycle *cycle);

/* Install a cycle schedule (re-records the iteration graphs with VMG_GRAPH,
 * so it may allocate).  Errors: VMG_EINVAL (null arguments, a field outside
 * its range or set for the wrong kind of plan), VMG_EHIP. */
vmg_status vmg_plan_set_cycle(vmg_plan *plan, const vmg_cycle *cycle);

/* Cycle-schedule autotuner (Sec. V: "more tunings of the code are needed").
 * Times complete solves of the given input (the arrays of vmg_solve; phi_work
 * is a device array of phi's layout holding the initial guess, from which every
 * trial starts, and receives the last trial's solution) to the plan's
 * tolerance for candidate schedules, by coordinate
 * search: nu1/nu2 over (1,1) .. (3,3), then the sweeps below the finest level
 * (as the finest, (1,1), (1,2), (2,1)), then inner cycles 1..6 and nu1/nu2
 * once more (mixed), then
 * coarsest sweeps {2, 4, 8, 16}, then the coarse tail on/off (periodic) or the
 * persistent launch size {512, 1024, 2048} (Dirichlet).  A candidate that does
 * not reach the tolerance within max_cycles is discarded.  The fastest
 * schedule is installed, returned in *best (may be NULL) with its median time
 * in *best_ms (may be NULL), and cached per (shape, precision, boundary kind,
 * grid count) in the process and in the file named by VMG_TUNE_CACHE, where a
 * later plan created with VMG_AUTOTUNE finds it (fields the caller set in
 * vmg_params, nu1/nu2 and inner_cycles, take precedence).  Allocates (graph
 * re-recording).  Errors: VMG_EINVAL (null plan, delta or phi_work; ghost
 * missing for Dirichlet plans), VMG_ENOCONV (no candidate converged), the
 * errors of vmg_solve. */
vmg_status vmg_plan_tune_cycle(vmg_plan *plan, const double *delta, const double *ghost, const double *source,
                               double *phi_work, vmg_cycle *best, double *best_ms);

/* Number of levels of a plan that run the fused red-black sweep (the finest
 * level and every coarser one above the single-launch coarse tail), i.e. the
 * levels vmg_plan_set_schedule and vmg_plan_schedule accept; -1 for NULL. */
int32_t vmg_plan_level_count(const vmg_plan *plan);

/* Install a sweep schedule on one level (Sec. V of the paper notes that the
 * code needed more tuning; this is how a caller reuses schedules the autotuner
 * found, or forces one): the fused sweep of level `level` then runs tiles of
 * 64 x tile_y cells marching z_chunk planes, with pipeline shape `pipe`: 0 =
 * the black phase one plane behind the red phase (two barriers per plane
 * step, three-plane LDS rings), 1 = two planes behind (one barrier, four-plane
 * rings); or, with pipe 2, the brick schedule: no z march, 8^3 bricks whose
 * rings are recomputed by every block, up to two sweeps per launch on a
 * coarser level of a periodic plan, one sweep per launch (the ghost shell as
 * the boundary) on any level of a Dirichlet batch (tile_y and z_chunk are then
 * only validated).
 * The schedule changes only the blocking of the same red-black update, not the
 * result's definition.  With VMG_GRAPH the iteration graphs are recorded again
 * (allocates).  Errors: VMG_EINVAL (null plan, level outside [0,
 * vmg_plan_level_count), tile_y not in {4, 8, 12, 16}, z_chunk odd or outside
 * [2, 1024], pipe not 0, 1 or 2, pipe 2 on the finest level of a periodic
 * plan), VMG_EHIP. */
vmg_status vmg_plan_set_schedule(vmg_plan *plan, int32_t level, int32_t tile_y, int32_t z_chunk, int32_t pipe);

/* The sweep schedule a level runs (host pointers, each may be NULL).
 * Errors: VMG_EINVAL (null plan, level outside [0, vmg_plan_level_count)). */
vmg_status vmg_plan_schedule(const vmg_plan *plan, int32_t level, int32_t *tile_y, int32_t *z_chunk,
                             int32_t *pipe);

#ifdef __cplusplus
}
#endif
#endif /* VMG_H */
