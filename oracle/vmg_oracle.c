/*
 * vmg_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, FP64 CPU implementation of the discrete problem solved by the
 * GPU library.  Only the test-suite, the smoke check and the CPU-baseline leg
 * of the benchmark may load it; the product path never does.  It shares no
 * code, header or table with the GPU path.
 *
 * What it computes (Li, Zhao & Koyama, "Exploring Vainshtein mechanism on
 * adaptively refined meshes"):
 *
 *   * Sec. III.A, Eq. (code_eqn): the brane-bending-mode equation in code
 *     units, written here with alpha_p = 3 beta a^4 / R_c^2 (the paper's
 *     "alpha") and the density term alpha_p * kappa * delta, where kappa is
 *     the source coefficient Omega_m a / beta.  The solver library's "alpha"
 *     is 1/alpha_p; this file converts once, in or_coeffs().
 *   * Sec. III.A, Eqs. (two_branch), (one_branch): operator splitting with
 *     constant w and the sign(alpha_p) branch of the quadratic root.
 *   * Sec. III.B: cell-centred finite differences, the discrete operator
 *     L^h phi = Lap_h phi - root(Sigma_ijk), the 19-point Sigma_ijk and the
 *     Newton-Gauss-Seidel update with dL/dphi.
 *   * Sec. III.C, Eq. (fine_grid_eqn) and the equations after it: full
 *     approximation scheme (FAS) V-cycles: residual d^h = L^h(phi^h) - f^h,
 *     coarse equation L^H(phi^H) = L^H(R phi^h) - R d^h, correction
 *     phi^h += P(phi^H - R phi^h).
 *
 * Readings where the paper is silent (each is also listed in the design notes):
 *   - periodic compatibility: the discrete nonlinear term does not sum to zero
 *     over a periodic grid, so the periodic equation carries a constant cbar on
 *     the f side: L^h(phi) + cbar = f, cbar = mean(f) - mean(L^h phi), and the
 *     gauge mean(phi) = 0 is imposed on the result;
 *   - negative discriminant: the square root is taken as 0 (vertex of the
 *     quadratic), i.e. root = -alpha_p / (2(1-w));
 *   - alpha = 0 (alpha_p infinite): the root tends to kappa*delta, the
 *     linearised (Poisson) limit of Sec. II.A, which is used directly;
 *   - R = average of the 8 children, P = cell-centred trilinear interpolation,
 *     coarse density = R(delta) ("by interpolation", Sec. III.C);
 *   - refinement boundary (Sec. III.C, IV.D): a one-cell ghost shell (faces and
 *     edges, no corners) around the n0*n1*n2 unknowns, values given;
 *   - coarse levels of a refinement (Sec. III.C only says they need suitable
 *     boundary conditions): the ghosts of a coarse level hold the restricted
 *     boundary values plus the odd reflection of the adjacent interior
 *     correction, so the coarse correction vanishes on the refinement's faces
 *     (the boundary values are fixed there); prolongation uses the same
 *     reflection.  A zero correction at the coarse ghost centres instead puts
 *     the boundary half a coarse cell too far out, and the V-cycle then slows
 *     down with every extra level;
 *   - Gauss-Seidel order (unspecified): lexicographic, x fastest.
 *
 * Array layout: every field handed in or out is x-fastest, unpadded
 * (index (k*n1 + j)*n0 + i).  Internally each level is stored padded,
 * (n0+2)*(n1+2)*(n2+2), so Dirichlet ghosts sit in the shell; periodic
 * levels ignore the shell and wrap indices instead.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int n[3];        /* cells per axis */
    int periodic;    /* 1: periodic wrap, 0: Dirichlet ghost shell */
    double h;        /* cell size */
} OGrid;

typedef struct {
    double alpha_p;  /* 3 beta a^4 / R_c^2 ; unused when linear */
    double dens;     /* coefficient of delta inside Sigma: alpha_p * kappa */
    double kappa;    /* used only in the linear limit */
    double w;        /* splitting constant (1/3 in the paper) */
    int linear;      /* alpha == 0 */
} OCoef;

static OCoef or_coeffs(double alpha, double kappa, double w) {
    OCoef c;
    c.w = w;
    c.kappa = kappa;
    c.linear = (alpha == 0.0);
    c.alpha_p = c.linear ? 0.0 : 1.0 / alpha;
    c.dens = c.alpha_p * kappa;
    return c;
}

static long ncells(const OGrid *g) { return (long)g->n[0] * g->n[1] * g->n[2]; }
static long npad(const OGrid *g) { return (long)(g->n[0] + 2) * (g->n[1] + 2) * (g->n[2] + 2); }

static long pidx(const OGrid *g, int i, int j, int k) {
    return ((long)(k + 1) * (g->n[1] + 2) + (j + 1)) * (g->n[0] + 2) + (i + 1);
}

static int wrap(int i, int n) {
    while (i < 0) i += n;
    while (i >= n) i -= n;
    return i;
}

/* value of a padded field at (i,j,k), i in [-1, n]; periodic grids wrap */
static double at(const OGrid *g, const double *u, int i, int j, int k) {
    if (g->periodic) {
        i = wrap(i, g->n[0]);
        j = wrap(j, g->n[1]);
        k = wrap(k, g->n[2]);
    }
    return u[pidx(g, i, j, k)];
}

/* The 19-point neighbourhood of a cell: v[a][b][c] = phi(i+a-1, j+b-1, k+c-1)
 * (the eight corners are not part of the stencil and are left unset). */
typedef struct { double v[3][3][3]; } Nbhd;

static void gather(const OGrid *g, const double *phi, int i, int j, int k, Nbhd *N) {
    for (int c = 0; c < 3; ++c)
        for (int b = 0; b < 3; ++b)
            for (int a = 0; a < 3; ++a) {
                const int off = (a != 1) + (b != 1) + (c != 1);
                N->v[a][b][c] = (off == 3) ? 0.0 : at(g, phi, i + a - 1, j + b - 1, k + c - 1);
            }
}

/* Everything the relaxation needs at one cell, from Sec. III.B:
 *   Sigma_{i,j,k} with splitting constant w (density term included),
 *   the sign(alpha_p) root of Eq. (one_branch),
 *   L^h phi = Lap_h phi - root, and dL^h/dphi_{i,j,k}. */
typedef struct { double sigma, disc, root, lap, L, dL; int guarded; } CellEval;

static CellEval cell_eval(const OGrid *g, const OCoef *c, const Nbhd *N, double delta_ijk) {
    CellEval e;
    const double h = g->h, h2 = h * h, h4 = h2 * h2, w = c->w;
    const double (*v)[3][3] = N->v;
    const double p = v[1][1][1];
    /* three-point second differences (h^2 times the second derivatives) */
    const double ax = v[2][1][1] + v[0][1][1] - 2.0 * p;
    const double ay = v[1][2][1] + v[1][0][1] - 2.0 * p;
    const double az = v[1][1][2] + v[1][1][0] - 2.0 * p;
    /* four-point cross differences (4 h^2 times the mixed derivatives) */
    const double bxy = v[2][2][1] + v[0][0][1] - v[2][0][1] - v[0][2][1];
    const double bxz = v[2][1][2] + v[0][1][0] - v[2][1][0] - v[0][1][2];
    const double byz = v[1][2][2] + v[1][0][0] - v[1][2][0] - v[1][0][2];
    const double lapsum = ax + ay + az;
    e.lap = lapsum / h2;
    double s = (1.0 - w) / h4 * (ax * ax + ay * ay + az * az);
    s -= 2.0 * w / h4 * ax * ay;
    s -= 2.0 * w / h4 * ax * az;
    s -= 2.0 * w / h4 * ay * az;
    s += (bxy * bxy + bxz * bxz + byz * byz) / (8.0 * h4);
    s += c->dens * delta_ijk;
    e.sigma = s;
    if (c->linear) {              /* alpha -> 0: the root tends to kappa*delta */
        e.disc = 1.0;
        e.guarded = 0;
        e.root = c->kappa * delta_ijk;
        e.L = e.lap - e.root;
        e.dL = -6.0 / h2;
        return e;
    }
    double dsc = c->alpha_p * c->alpha_p + 4.0 * (1.0 - w) * s;
    e.disc = dsc;
    e.guarded = dsc < 0.0;
    if (dsc < 0.0) dsc = 0.0;     /* vertex of the quadratic */
    const double sgn = c->alpha_p > 0.0 ? 1.0 : -1.0;
    e.root = (-c->alpha_p + sgn * sqrt(dsc)) / (2.0 * (1.0 - w));
    e.L = e.lap - e.root;
    if (dsc > 0.0)
        e.dL = -6.0 / h2 + sgn * 4.0 * (1.0 - 3.0 * w) / (h4 * sqrt(dsc)) * lapsum;
    else
        e.dL = -6.0 / h2;         /* clamped root does not depend on phi */
    return e;
}

static CellEval eval_at(const OGrid *g, const OCoef *c, const double *phi, const double *delta,
                        int i, int j, int k) {
    Nbhd N;
    gather(g, phi, i, j, k, &N);
    return cell_eval(g, c, &N, at(g, delta, i, j, k));
}

/* Sec. III.B: L^h phi_{i,j,k} */
static double Lh(const OGrid *g, const OCoef *c, const double *phi, const double *delta,
                 int i, int j, int k, double *root_out, int *guarded) {
    const CellEval e = eval_at(g, c, phi, delta, i, j, k);
    if (root_out) *root_out = e.root;
    if (guarded) *guarded = e.guarded;
    return e.L;
}

/* ------------------------------------------------------------------------- */
/* level storage                                                              */
/* ------------------------------------------------------------------------- */
typedef struct {
    OGrid g;
    double *phi, *phiold, *f, *delta, *d;  /* all padded */
} OLevel;

static void level_alloc(OLevel *L, const OGrid *g) {
    L->g = *g;
    const long np = npad(g);
    L->phi = calloc(np, sizeof(double));
    L->phiold = calloc(np, sizeof(double));
    L->f = calloc(np, sizeof(double));
    L->delta = calloc(np, sizeof(double));
    L->d = calloc(np, sizeof(double));
}

static void level_free(OLevel *L) {
    free(L->phi); free(L->phiold); free(L->f); free(L->delta); free(L->d);
}

static void unpack(const OGrid *g, const double *src, double *pad) {
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i)
                pad[pidx(g, i, j, k)] = src[((long)k * g->n[1] + j) * g->n[0] + i];
}

static void pack(const OGrid *g, const double *pad, double *dst) {
    for (int k = 0; k < g->n[2]; ++k)
        for (int j = 0; j < g->n[1]; ++j)
            for (int i = 0; i < g->n[0]; ++i)
                dst[((long)k * g->n[1] + j) * g->n[0] + i] = pad[pidx(g, i, j, k)];
}

/* Ghost shell, compact order: faces x-,x+ (j fastest, then k), y-,y+ (i, k),
 * z-,z+ (i, j); then edges along x: (y-,z-),(y+,z-),(y-,z+),(y+,z+) (i);
 * along y: (x-,z-),(x+,z-),(x-,z+),(x+,z+) (j); along z: (x-,y-),(x+,y-),
 * (x-,y+),(x+,y+) (k). */
static long ghost_count(const int n[3]) {
    return 2L * ((long)n[1] * n[2] + (long)n[0] * n[2] + (long)n[0] * n[1]) + 4L * (n[0] + n[1] + n[2]);
}

static void ghosts_to_pad(const OGrid *g, const double *ghost, double *pad) {
    const int n0 = g->n[0], n1 = g->n[1], n2 = g->n[2];
    long q = 0;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < n2; ++k)
            for (int j = 0; j < n1; ++j) pad[pidx(g, s ? n0 : -1, j, k)] = ghost[q++];
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < n2; ++k)
            for (int i = 0; i < n0; ++i) pad[pidx(g, i, s ? n1 : -1, k)] = ghost[q++];
    for (int s = 0; s < 2; ++s)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) pad[pidx(g, i, j, s ? n2 : -1)] = ghost[q++];
    for (int e = 0; e < 4; ++e)
        for (int i = 0; i < n0; ++i) pad[pidx(g, i, (e & 1) ? n1 : -1, (e & 2) ? n2 : -1)] = ghost[q++];
    for (int e = 0; e < 4; ++e)
        for (int j = 0; j < n1; ++j) pad[pidx(g, (e & 1) ? n0 : -1, j, (e & 2) ? n2 : -1)] = ghost[q++];
    for (int e = 0; e < 4; ++e)
        for (int k = 0; k < n2; ++k) pad[pidx(g, (e & 1) ? n0 : -1, (e & 2) ? n1 : -1, k)] = ghost[q++];
}

/* ------------------------------------------------------------------------- */
/* residual, cbar                                                             */
/* ------------------------------------------------------------------------- */

/* cbar = mean(f) - mean(L^h phi) on periodic levels, 0 on Dirichlet levels */
/* Compensated (Neumaier) summation: the grid sums below add up to 1e8 terms
 * that cancel (the Laplacian sums to zero on a periodic grid), where a plain
 * running sum would lose the digits that cbar and the residual norm need. */
typedef struct { double s, c; } KSum;

static void ks_add(KSum *k, double x) {
    const double t = k->s + x;
    if (fabs(k->s) >= fabs(x)) k->c += (k->s - t) + x;
    else k->c += (x - t) + k->s;
    k->s = t;
}

static double ks_val(const KSum *k) { return k->s + k->c; }

static double compat_const(const OLevel *L, const OCoef *c) {
    if (!L->g.periodic) return 0.0;
    KSum sf = {0.0, 0.0}, sl = {0.0, 0.0};
    for (int k = 0; k < L->g.n[2]; ++k)
        for (int j = 0; j < L->g.n[1]; ++j)
            for (int i = 0; i < L->g.n[0]; ++i) {
                ks_add(&sf, L->f[pidx(&L->g, i, j, k)]);
                ks_add(&sl, Lh(&L->g, c, L->phi, L->delta, i, j, k, NULL, NULL));
            }
    return (ks_val(&sf) - ks_val(&sl)) / (double)ncells(&L->g);
}

/* d = L^h phi + cbar - f; returns sum d^2; optional sums of the root and guard count */
static double residual(OLevel *L, const OCoef *c, double cbar, double *sum_root, long *nguard) {
    KSum s2 = {0.0, 0.0}, sr = {0.0, 0.0};
    long ng = 0;
    for (int k = 0; k < L->g.n[2]; ++k)
        for (int j = 0; j < L->g.n[1]; ++j)
            for (int i = 0; i < L->g.n[0]; ++i) {
                double r;
                int gd;
                const long p = pidx(&L->g, i, j, k);
                const double v = Lh(&L->g, c, L->phi, L->delta, i, j, k, &r, &gd) + cbar - L->f[p];
                L->d[p] = v;
                ks_add(&s2, v * v);
                ks_add(&sr, r);
                ng += gd;
            }
    if (sum_root) *sum_root = ks_val(&sr);
    if (nguard) *nguard = ng;
    return ks_val(&s2);
}

/* ------------------------------------------------------------------------- */
/* relaxation: lexicographic Newton-Gauss-Seidel (Sec. III.B)                 */
/* ------------------------------------------------------------------------- */
/* Kink cells (reading: the paper does not discuss relaxation at the guard).
 * Near D = 0, with D = disc / alpha_p^2 the normalised discriminant, the
 * root's slope 1/sqrt(D) couples a cell so strongly to its neighbours that
 * plain Gauss-Seidel updates can settle into a two-sweep oscillation across
 * D = 0 (one sweep on the clamped side, the next on the steep side).  That
 * coupling grows like 1 / (h^2 sqrt|D|), so the update is under-relaxed by
 * w = min(1, max(KINK_WMIN, KINK_K h^2 sqrt|D|)); w = 1 wherever
 * KINK_K h^2 sqrt|D| >= 1.  The fixed point, i.e. the discrete solution, is
 * unchanged. */
#define KINK_K (50.0 * 65536.0)
#define KINK_WMIN 0.01

static double update_weight(const OGrid *g, const OCoef *c, const CellEval *e) {
    if (c->linear) return 1.0;
    const double w = KINK_K * g->h * g->h * sqrt(fabs(e->disc) / (c->alpha_p * c->alpha_p));
    return w < 1.0 ? fmax(w, KINK_WMIN) : 1.0;
}

static void relax(OLevel *L, const OCoef *c, int sweeps) {
    for (int s = 0; s < sweeps; ++s) {
        const double cbar = compat_const(L, c);
        for (int k = 0; k < L->g.n[2]; ++k)
            for (int j = 0; j < L->g.n[1]; ++j)
                for (int i = 0; i < L->g.n[0]; ++i) {
                    const long p = pidx(&L->g, i, j, k);
                    const CellEval e = eval_at(&L->g, c, L->phi, L->delta, i, j, k);
                    L->phi[p] -= update_weight(&L->g, c, &e) * (e.L + cbar - L->f[p]) / e.dL;
                }
    }
}

/* ------------------------------------------------------------------------- */
/* restriction / prolongation (Sec. III.C)                                    */
/* ------------------------------------------------------------------------- */
static double child_mean(const OGrid *fg, const double *u, int I, int J, int K) {
    double s = 0.0;
    for (int dk = 0; dk < 2; ++dk)
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) s += u[pidx(fg, 2 * I + di, 2 * J + dj, 2 * K + dk)];
    return s / 8.0;
}

static void restrict_field(const OGrid *fg, const double *uf, const OGrid *cg, double *uc) {
    for (int K = 0; K < cg->n[2]; ++K)
        for (int J = 0; J < cg->n[1]; ++J)
            for (int I = 0; I < cg->n[0]; ++I) uc[pidx(cg, I, J, K)] = child_mean(fg, uf, I, J, K);
}

/* coarse Dirichlet ghosts: mean of the fine ghost cells lying inside each coarse ghost cell */
static void restrict_ghosts(const OGrid *fg, const double *uf, const OGrid *cg, double *uc) {
    for (int K = -1; K <= cg->n[2]; ++K)
        for (int J = -1; J <= cg->n[1]; ++J)
            for (int I = -1; I <= cg->n[0]; ++I) {
                const int outside = (I < 0 || I >= cg->n[0]) + (J < 0 || J >= cg->n[1]) + (K < 0 || K >= cg->n[2]);
                if (outside == 0 || outside == 3) continue;
                double s = 0.0;
                int cnt = 0;
                for (int dk = 0; dk < 2; ++dk)
                    for (int dj = 0; dj < 2; ++dj)
                        for (int di = 0; di < 2; ++di) {
                            const int i = 2 * I + di, j = 2 * J + dj, k = 2 * K + dk;
                            if (i < -1 || i > fg->n[0] || j < -1 || j > fg->n[1] || k < -1 || k > fg->n[2]) continue;
                            const int o = (i < 0 || i >= fg->n[0]) + (j < 0 || j >= fg->n[1]) + (k < 0 || k >= fg->n[2]);
                            if (o == 0 || o == 3) continue;
                            s += uf[pidx(fg, i, j, k)];
                            ++cnt;
                        }
                uc[pidx(cg, I, J, K)] = cnt ? s / cnt : 0.0;
            }
}

/* Reflect an index one cell outside [0, n) back inside, flipping *sign. */
static int reflect(int i, int n, int *sign) {
    if (i < 0) { *sign = -*sign; return 0; }
    if (i >= n) { *sign = -*sign; return n - 1; }
    return i;
}

/* Correction phi - phiold at (i,j,k) of a Dirichlet level, ghosts included:
 * outside the grid it is minus (per crossed face) the value at the mirror cell. */
static double dir_corr(const OLevel *C, int i, int j, int k) {
    int sg = 1;
    const int a = reflect(i, C->g.n[0], &sg), b = reflect(j, C->g.n[1], &sg), e = reflect(k, C->g.n[2], &sg);
    const long p = pidx(&C->g, a, b, e);
    return sg * (C->phi[p] - C->phiold[p]);
}

/* Coarse Dirichlet level: ghosts = restricted boundary values (kept in the
 * ghosts of phiold) + reflected interior correction. */
static void refresh_ghosts(OLevel *C) {
    const OGrid *g = &C->g;
    for (int k = -1; k <= g->n[2]; ++k)
        for (int j = -1; j <= g->n[1]; ++j)
            for (int i = -1; i <= g->n[0]; ++i) {
                const int o = (i < 0 || i >= g->n[0]) + (j < 0 || j >= g->n[1]) + (k < 0 || k >= g->n[2]);
                if (o == 0 || o == 3) continue;
                const long p = pidx(g, i, j, k);
                C->phi[p] = C->phiold[p] + dir_corr(C, i, j, k);
            }
}

/* fine += P(coarse correction); on a Dirichlet grid the correction outside is
 * the reflection of the interior one */
static void prolong_add(const OLevel *C, OLevel *F) {
    const OGrid *cg = &C->g, *fg = &F->g;
    for (int k = 0; k < fg->n[2]; ++k)
        for (int j = 0; j < fg->n[1]; ++j)
            for (int i = 0; i < fg->n[0]; ++i) {
                const int I = i / 2, J = j / 2, K = k / 2;
                const int si = (i & 1) ? 1 : -1, sj = (j & 1) ? 1 : -1, sk = (k & 1) ? 1 : -1;
                double acc = 0.0;
                for (int a = 0; a < 2; ++a)
                    for (int b = 0; b < 2; ++b)
                        for (int e = 0; e < 2; ++e) {
                            const double wgt = (a ? 0.25 : 0.75) * (b ? 0.25 : 0.75) * (e ? 0.25 : 0.75);
                            int ii = I + a * si, jj = J + b * sj, kk = K + e * sk;
                            double corr;
                            if (cg->periodic)
                                corr = at(cg, C->phi, ii, jj, kk) - at(cg, C->phiold, ii, jj, kk);
                            else
                                corr = dir_corr(C, ii, jj, kk);
                            acc += wgt * corr;
                        }
                F->phi[pidx(fg, i, j, k)] += acc;
            }
}

/* ------------------------------------------------------------------------- */
/* hierarchy and V-cycle                                                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nlev;
    OLevel lev[24];
    OCoef c;
    int nu1, nu2, ncoarse;
} OHier;

static int can_coarsen(const OGrid *g) {
    const int minc = g->periodic ? 4 : 2;
    for (int d = 0; d < 3; ++d)
        if ((g->n[d] & 1) || g->n[d] / 2 < minc) return 0;
    return 1;
}

static void hier_build(OHier *H, const OGrid *g0) {
    H->nlev = 0;
    OGrid g = *g0;
    for (;;) {
        level_alloc(&H->lev[H->nlev++], &g);
        if (!can_coarsen(&g) || H->nlev == 24) break;
        g.n[0] /= 2; g.n[1] /= 2; g.n[2] /= 2; g.h *= 2.0;
    }
}

static void hier_free(OHier *H) {
    for (int l = 0; l < H->nlev; ++l) level_free(&H->lev[l]);
}

/* Sweeps on level l; a coarse Dirichlet level refreshes its ghosts after each. */
static void relax_level(OHier *H, int l, int sweeps) {
    OLevel *F = &H->lev[l];
    const int refresh = l > 0 && !F->g.periodic;
    for (int s = 0; s < sweeps; ++s) {
        relax(F, &H->c, 1);
        if (refresh) refresh_ghosts(F);
    }
}

static void vcycle(OHier *H, int l) {
    OLevel *F = &H->lev[l];
    if (l == H->nlev - 1) {
        relax_level(H, l, H->ncoarse);
        return;
    }
    OLevel *C = &H->lev[l + 1];
    relax_level(H, l, H->nu1);
    const double cbar = compat_const(F, &H->c);
    residual(F, &H->c, cbar, NULL, NULL);
    restrict_field(&F->g, F->phi, &C->g, C->phi);
    if (C->g.periodic) {
        memcpy(C->phiold, C->phi, sizeof(double) * npad(&C->g));
    } else {
        /* interior only: the ghosts of phiold keep the restricted boundary values */
        for (int K = 0; K < C->g.n[2]; ++K)
            for (int J = 0; J < C->g.n[1]; ++J)
                for (int I = 0; I < C->g.n[0]; ++I) C->phiold[pidx(&C->g, I, J, K)] = C->phi[pidx(&C->g, I, J, K)];
        refresh_ghosts(C);
    }
    /* f^H = L^H(R phi^h) - R d^h (the coarse periodic constant drops out: only
     * f^H - mean(f^H) matters to the projected coarse equation) */
    restrict_field(&F->g, F->d, &C->g, C->d);
    for (int K = 0; K < C->g.n[2]; ++K)
        for (int J = 0; J < C->g.n[1]; ++J)
            for (int I = 0; I < C->g.n[0]; ++I) {
                const long p = pidx(&C->g, I, J, K);
                C->f[p] = Lh(&C->g, &H->c, C->phi, C->delta, I, J, K, NULL, NULL) - C->d[p];
            }
    vcycle(H, l + 1);
    prolong_add(C, F);
    relax_level(H, l, H->nu2);
}

/* ------------------------------------------------------------------------- */
/* exported entry points (called from Python through ctypes)                  */
/* ------------------------------------------------------------------------- */

/* Residual of a given phi on one grid.  d_out (may be NULL) receives d =
 * L^h phi + cbar - f; stats[0]=rms, [1]=cbar, [2]=mean root, [3]=guard count. */
int or_residual(const int n[3], int periodic, double h, double alpha, double kappa, double w,
                const double *delta, const double *ghost, const double *source, const double *phi,
                double *d_out, double *stats) {
    OGrid g = {{n[0], n[1], n[2]}, periodic, h};
    OCoef c = or_coeffs(alpha, kappa, w);
    OLevel L;
    level_alloc(&L, &g);
    unpack(&g, delta, L.delta);
    unpack(&g, phi, L.phi);
    if (source) unpack(&g, source, L.f);
    if (!periodic && ghost) ghosts_to_pad(&g, ghost, L.phi);
    const double cbar = compat_const(&L, &c);
    double sr;
    long ng;
    const double s2 = residual(&L, &c, cbar, &sr, &ng);
    if (d_out) pack(&g, L.d, d_out);
    stats[0] = sqrt(s2 / (double)ncells(&g));
    stats[1] = cbar;
    stats[2] = sr / (double)ncells(&g);
    stats[3] = (double)ng;
    level_free(&L);
    return 0;
}

/* Solve L^h phi (+ cbar) = f with FAS V(nu1,nu2) cycles of lexicographic
 * Newton-GS until rms <= tol, stagnation (no 2x drop over 4 cycles) or
 * max_cycles.  phi is the initial guess on entry and the solution on exit
 * (periodic: mean removed).  info[0]=rms, [1]=cycles, [2]=cbar, [3]=guard count. */
int or_solve(const int n[3], int periodic, double h, double alpha, double kappa, double w,
             const double *delta, const double *ghost, const double *source, double *phi,
             double tol, int max_cycles, int nu1, int nu2, double *info) {
    OGrid g = {{n[0], n[1], n[2]}, periodic, h};
    OHier H;
    H.c = or_coeffs(alpha, kappa, w);
    H.nu1 = nu1;
    H.nu2 = nu2;
    H.ncoarse = 60;
    hier_build(&H, &g);
    OLevel *F = &H.lev[0];
    unpack(&g, delta, F->delta);
    unpack(&g, phi, F->phi);
    if (source) unpack(&g, source, F->f);
    if (!periodic && ghost) ghosts_to_pad(&g, ghost, F->phi);
    for (int l = 1; l < H.nlev; ++l) {
        restrict_field(&H.lev[l - 1].g, H.lev[l - 1].delta, &H.lev[l].g, H.lev[l].delta);
        if (!periodic) {
            restrict_ghosts(&H.lev[l - 1].g, H.lev[l - 1].phi, &H.lev[l].g, H.lev[l].phi);
            memcpy(H.lev[l].phiold, H.lev[l].phi, sizeof(double) * npad(&H.lev[l].g));
        }
    }
    double rms = 0.0, best = 1e300, hist[8] = {1e300, 1e300, 1e300, 1e300, 1e300, 1e300, 1e300, 1e300};
    int cyc = 0;
    for (;;) {
        const double cbar = compat_const(F, &H.c);
        rms = sqrt(residual(F, &H.c, cbar, NULL, NULL) / (double)ncells(&g));
        if (!(rms == rms)) break;
        if (rms <= tol || cyc >= max_cycles) break;
        /* stagnated at the rounding floor: less than 10% gained over 8 cycles (a
         * slow nonlinear start phase still gains more than that) */
        if (cyc >= 8 && rms > 0.9 * hist[cyc % 8]) break;
        hist[cyc % 8] = rms;
        if (rms < best) best = rms;
        vcycle(&H, 0);
        ++cyc;
    }
    if (periodic) {
        KSum ms = {0.0, 0.0};
        for (int k = 0; k < g.n[2]; ++k)
            for (int j = 0; j < g.n[1]; ++j)
                for (int i = 0; i < g.n[0]; ++i) ks_add(&ms, F->phi[pidx(&g, i, j, k)]);
        const double m = ks_val(&ms) / (double)ncells(&g);
        for (int k = 0; k < g.n[2]; ++k)
            for (int j = 0; j < g.n[1]; ++j)
                for (int i = 0; i < g.n[0]; ++i) F->phi[pidx(&g, i, j, k)] -= m;
    }
    const double cbar = compat_const(F, &H.c);
    double sr;
    long ng;
    rms = sqrt(residual(F, &H.c, cbar, &sr, &ng) / (double)ncells(&g));
    pack(&g, F->phi, phi);
    info[0] = rms;
    info[1] = cyc;
    info[2] = cbar;
    info[3] = (double)ng;
    hier_free(&H);
    return 0;
}

/* Run exactly `sweeps` lexicographic Newton-GS sweeps (no multigrid). */
int or_relax(const int n[3], int periodic, double h, double alpha, double kappa, double w,
             const double *delta, const double *ghost, const double *source, double *phi, int sweeps) {
    OGrid g = {{n[0], n[1], n[2]}, periodic, h};
    OCoef c = or_coeffs(alpha, kappa, w);
    OLevel L;
    level_alloc(&L, &g);
    unpack(&g, delta, L.delta);
    unpack(&g, phi, L.phi);
    if (source) unpack(&g, source, L.f);
    if (!periodic && ghost) ghosts_to_pad(&g, ghost, L.phi);
    relax(&L, &c, sweeps);
    pack(&g, L.phi, phi);
    level_free(&L);
    return 0;
}

/* One cell (Sec. III.B): out[0]=L^h phi, [1]=dL^h/dphi, [2]=Sigma_ijk, [3]=root */
int or_cell_operator(const int n[3], int periodic, double h, double alpha, double kappa, double w,
                     const double *delta, const double *ghost, const double *phi,
                     int i, int j, int k, double *out) {
    OGrid g = {{n[0], n[1], n[2]}, periodic, h};
    OCoef c = or_coeffs(alpha, kappa, w);
    OLevel L;
    level_alloc(&L, &g);
    unpack(&g, delta, L.delta);
    unpack(&g, phi, L.phi);
    if (!periodic && ghost) ghosts_to_pad(&g, ghost, L.phi);
    const CellEval e = eval_at(&g, &c, L.phi, L.delta, i, j, k);
    out[0] = e.L;
    out[1] = e.dL;
    out[2] = e.sigma;
    out[3] = e.root;
    level_free(&L);
    return 0;
}

/* Trilinear interpolation of a cell-centred periodic parent field (np0,np1,np2
 * cells of size H) at the centre of patch cell (i,j,k); the patch has cells of
 * size h and its cell (0,0,0) starts at origin*h (Sec. III.C, IV.D: values on a
 * refinement are interpolated from the coarser level). */
static double parent_trilinear(const int np_[3], double H, const double *parent, double h, const int origin[3],
                               int i, int j, int k) {
    const int ii[3] = {i, j, k};
    int base[3];
    double t[3];
    for (int d = 0; d < 3; ++d) {
        const double x = (origin[d] + ii[d] + 0.5) * h;        /* box coordinate */
        const double u = x / H - 0.5;                            /* parent index space */
        const double fl = floor(u);
        base[d] = (int)fl;
        t[d] = u - fl;
    }
    double v = 0.0;
    for (int c2 = 0; c2 < 2; ++c2)
        for (int c1 = 0; c1 < 2; ++c1)
            for (int c0 = 0; c0 < 2; ++c0) {
                const double wgt = (c0 ? t[0] : 1 - t[0]) * (c1 ? t[1] : 1 - t[1]) * (c2 ? t[2] : 1 - t[2]);
                const int I = wrap(base[0] + c0, np_[0]), J = wrap(base[1] + c1, np_[1]), K = wrap(base[2] + c2, np_[2]);
                v += wgt * parent[((long)K * np_[1] + J) * np_[0] + I];
            }
    return v;
}

/* Initial guess on a refinement: the parent interpolated at every patch cell
 * centre; output x-fastest n0*n1*n2. */
int or_fill_interior(const int np_[3], double H, const double *parent, const int n[3], double h,
                     const int origin[3], double *phi) {
    long q = 0;
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) phi[q++] = parent_trilinear(np_, H, parent, h, origin, i, j, k);
    return 0;
}

/* Refinement boundary values: the same interpolation at the centres of a
 * patch's ghost cells, output in the compact ghost order. */
int or_fill_ghosts(const int np_[3], double H, const double *parent, const int n[3], double h,
                   const int origin[3], double *ghost) {
    OGrid g = {{n[0], n[1], n[2]}, 0, h};
    double *pad = calloc(npad(&g), sizeof(double));
    for (int k = -1; k <= n[2]; ++k)
        for (int j = -1; j <= n[1]; ++j)
            for (int i = -1; i <= n[0]; ++i) {
                const int o = (i < 0 || i >= n[0]) + (j < 0 || j >= n[1]) + (k < 0 || k >= n[2]);
                if (o == 0 || o == 3) continue;
                pad[pidx(&g, i, j, k)] = parent_trilinear(np_, H, parent, h, origin, i, j, k);
            }
    /* pad -> compact */
    const int n0 = n[0], n1 = n[1], n2 = n[2];
    long q = 0;
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < n2; ++k)
            for (int j = 0; j < n1; ++j) ghost[q++] = pad[pidx(&g, s ? n0 : -1, j, k)];
    for (int s = 0; s < 2; ++s)
        for (int k = 0; k < n2; ++k)
            for (int i = 0; i < n0; ++i) ghost[q++] = pad[pidx(&g, i, s ? n1 : -1, k)];
    for (int s = 0; s < 2; ++s)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) ghost[q++] = pad[pidx(&g, i, j, s ? n2 : -1)];
    for (int e = 0; e < 4; ++e)
        for (int i = 0; i < n0; ++i) ghost[q++] = pad[pidx(&g, i, (e & 1) ? n1 : -1, (e & 2) ? n2 : -1)];
    for (int e = 0; e < 4; ++e)
        for (int j = 0; j < n1; ++j) ghost[q++] = pad[pidx(&g, (e & 1) ? n0 : -1, j, (e & 2) ? n2 : -1)];
    for (int e = 0; e < 4; ++e)
        for (int k = 0; k < n2; ++k) ghost[q++] = pad[pidx(&g, (e & 1) ? n0 : -1, (e & 2) ? n1 : -1, k)];
    free(pad);
    return (int)(q == ghost_count(n) ? 0 : -1);
}

long or_ghost_count(const int n[3]) { return ghost_count(n); }

/* ------------------------------------------------------------------------- */
/* total potential and force (Sec. II.B, Sec. III.B)                          */
/* ------------------------------------------------------------------------- */
/* On a periodic n[0] x n[1] x n[2] grid (x fastest) of cell size h: the total
 * potential Psi = phi_N + phi/2 of the model, and the acceleration -grad Psi
 * by the central difference (Psi_{i+1} - Psi_{i-1}) / (2h) along each axis,
 * with periodic neighbours.  psi and g[3 * N] (gx, then gy, then gz) are
 * written; phi_N solves the Newtonian Poisson equation.  Returns 0. */
int or_total_force(const int n[3], double h, const double *phi_n, const double *phi, double *psi, double *g) {
    const int n0 = n[0], n1 = n[1], n2 = n[2];
    const long N = (long)n0 * n1 * n2;
    for (long e = 0; e < N; ++e) psi[e] = phi_n[e] + 0.5 * phi[e];
    for (int k = 0; k < n2; ++k)
        for (int j = 0; j < n1; ++j)
            for (int i = 0; i < n0; ++i) {
                const long e = ((long)k * n1 + j) * n0 + i;
                const long xp = ((long)k * n1 + j) * n0 + wrap(i + 1, n0);
                const long xm = ((long)k * n1 + j) * n0 + wrap(i - 1, n0);
                const long yp = ((long)k * n1 + wrap(j + 1, n1)) * n0 + i;
                const long ym = ((long)k * n1 + wrap(j - 1, n1)) * n0 + i;
                const long zp = ((long)wrap(k + 1, n2) * n1 + j) * n0 + i;
                const long zm = ((long)wrap(k - 1, n2) * n1 + j) * n0 + i;
                g[e] = -(psi[xp] - psi[xm]) / (2.0 * h);
                g[N + e] = -(psi[yp] - psi[ym]) / (2.0 * h);
                g[2 * N + e] = -(psi[zp] - psi[zm]) / (2.0 * h);
            }
    return 0;
}

/* ------------------------------------------------------------------------- */
/* truncation-error estimate (Sec. III.C)                                     */
/* ------------------------------------------------------------------------- */
/* tau^h = L^H(R phi^h) - R L^h(phi^h) on the next coarser level of a grid with
 * even sides (coarse density R delta), written unpadded to tau (n/2 cells per
 * axis).
 * Periodic: *rms = RMS of tau with its mean removed (a constant carries no
 * information on a periodic grid).
 * Dirichlet (ghost = the grid's boundary values in the compact order of
 * ghosts_to_pad): the coarse operator reads the restricted boundary values (mean
 * of the fine ghost cells inside each coarse ghost cell), the values a coarse
 * level of the V-cycle holds when its right-hand side is formed; *rms = plain RMS
 * of tau (no free constant on such a grid).
 * Returns 0, or -1 for odd sides or a Dirichlet grid without ghosts. */
int or_truncation_error(const int n[3], int periodic, double h, double alpha, double kappa, double w,
                        const double *delta, const double *ghost, const double *phi, double *tau, double *rms) {
    if ((n[0] & 1) || (n[1] & 1) || (n[2] & 1) || (!periodic && !ghost)) return -1;
    const OGrid gf = {{n[0], n[1], n[2]}, periodic, h};
    const OGrid gc = {{n[0] / 2, n[1] / 2, n[2] / 2}, periodic, 2.0 * h};
    const OCoef c = or_coeffs(alpha, kappa, w);
    double *pf = calloc(npad(&gf), sizeof(double)), *df = calloc(npad(&gf), sizeof(double));
    double *lf = calloc(npad(&gf), sizeof(double));
    double *pc = calloc(npad(&gc), sizeof(double)), *dc = calloc(npad(&gc), sizeof(double));
    unpack(&gf, phi, pf);
    unpack(&gf, delta, df);
    if (!periodic) {
        ghosts_to_pad(&gf, ghost, pf);
        restrict_ghosts(&gf, pf, &gc, pc);
    }
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) lf[pidx(&gf, i, j, k)] = Lh(&gf, &c, pf, df, i, j, k, NULL, NULL);
    restrict_field(&gf, pf, &gc, pc);
    restrict_field(&gf, df, &gc, dc);
    KSum s1 = {0.0, 0.0}, s2 = {0.0, 0.0};
    long q = 0;
    for (int K = 0; K < gc.n[2]; ++K)
        for (int J = 0; J < gc.n[1]; ++J)
            for (int I = 0; I < gc.n[0]; ++I, ++q) {
                const double t = Lh(&gc, &c, pc, dc, I, J, K, NULL, NULL) - child_mean(&gf, lf, I, J, K);
                tau[q] = t;
                ks_add(&s1, t);
                ks_add(&s2, t * t);
            }
    const double N = (double)q, m = periodic ? ks_val(&s1) / N : 0.0;
    *rms = sqrt(fmax(ks_val(&s2) / N - m * m, 0.0));
    free(pf); free(df); free(lf); free(pc); free(dc);
    return 0;
}

/* ------------------------------------------------------------------------- */
/* mass assignment: particles -> density contrast on the grid                 */
/* ------------------------------------------------------------------------- */
/* Unit-mass particles at pos[3*p + a] in [0, 1) (box units, a = x, y, z) on a
 * periodic unit box of n[0] x n[1] x n[2] cells (cell centres at (i + 1/2)/n).
 * With u = pos * n in cell units along an axis:
 *   scheme 1, cloud in cell: u' = u - 1/2, weight 1 - t to cell floor(u') and t
 *     to the next, t = u' - floor(u');
 *   scheme 2, triangular-shaped cloud (the scheme of Sec. VI): nearest cell
 *     c = floor(u), d = u - (c + 1/2); weights (1/2 - d)^2 / 2, 3/4 - d^2 and
 *     (1/2 + d)^2 / 2 to cells c - 1, c, c + 1.
 * The 3-D weight is the product of the axes' weights (periodic cells).
 * A coordinate outside [0, 1) is taken modulo 1 first (periodic box); a particle
 * with a non-finite coordinate deposits nothing but still counts in the mean.
 * delta = rho / mean(rho) - 1 with mean(rho) = n_particles / n_cells.
 * Returns 0, or -1 for an unknown scheme or n_particles < 1. */
int or_mass_assign(const double *pos, long np, const int n[3], int scheme, double *delta) {
    if ((scheme != 1 && scheme != 2) || np < 1) return -1;
    const int m = scheme == 1 ? 2 : 3;
    const long N = (long)n[0] * n[1] * n[2];
    for (long e = 0; e < N; ++e) delta[e] = 0.0;
    for (long p = 0; p < np; ++p) {
        int c[3][3];
        double w[3][3];
        if (!isfinite(pos[3 * p]) || !isfinite(pos[3 * p + 1]) || !isfinite(pos[3 * p + 2])) continue;
        for (int a = 0; a < 3; ++a) {
            const double u = (pos[3 * p + a] - floor(pos[3 * p + a])) * n[a];
            if (scheme == 1) {
                const double f = floor(u - 0.5);
                const double t = (u - 0.5) - f;
                c[a][0] = wrap((int)f, n[a]);
                c[a][1] = wrap((int)f + 1, n[a]);
                w[a][0] = 1.0 - t;
                w[a][1] = t;
            } else {
                const double f = floor(u);
                const double d = u - (f + 0.5);
                for (int q = 0; q < 3; ++q) c[a][q] = wrap((int)f + q - 1, n[a]);
                w[a][0] = 0.5 * (0.5 - d) * (0.5 - d);
                w[a][1] = 0.75 - d * d;
                w[a][2] = 0.5 * (0.5 + d) * (0.5 + d);
            }
        }
        for (int qz = 0; qz < m; ++qz)
            for (int qy = 0; qy < m; ++qy)
                for (int qx = 0; qx < m; ++qx)
                    delta[((long)c[2][qz] * n[1] + c[1][qy]) * n[0] + c[0][qx]] += w[0][qx] * w[1][qy] * w[2][qz];
    }
    const double scale = (double)N / (double)np;
    for (long e = 0; e < N; ++e) delta[e] = delta[e] * scale - 1.0;
    return 0;
}

/* The same assignment onto a refinement region: n[0] x n[1] x n[2] cells of
 * size h whose cell (0,0,0) corner sits at corner[] (box units), not periodic.
 * Along an axis a particle's offset from the corner is taken modulo 1 into
 * [0, 1) and moved to (offset - 1) when it lies more than n h + 2h past the
 * corner, so a particle just below the corner counts there; with n h <= 1 - 4h
 * at most one periodic image of a particle reaches the region.  In cell units
 * u = offset / h the weights are those of or_mass_assign; contributions to
 * cells outside the region are dropped.  delta = mass / mean_count - 1, with
 * mean_count the box's mean number of particles per cell of this size.
 * Returns 0, or -1 for bad arguments. */
int or_mass_assign_region(const double *pos, long np, const int n[3], double h, const double corner[3],
                          double mean_count, int scheme, double *delta) {
    if ((scheme != 1 && scheme != 2) || np < 0 || !(h > 0.0) || !(mean_count > 0.0)) return -1;
    for (int a = 0; a < 3; ++a)
        if (n[a] < 1 || n[a] * h > 1.0 - 4.0 * h) return -1;
    const int m = scheme == 1 ? 2 : 3;
    const long N = (long)n[0] * n[1] * n[2];
    for (long e = 0; e < N; ++e) delta[e] = 0.0;
    for (long p = 0; p < np; ++p) {
        int c[3][3];
        double w[3][3];
        if (!isfinite(pos[3 * p]) || !isfinite(pos[3 * p + 1]) || !isfinite(pos[3 * p + 2])) continue;
        for (int a = 0; a < 3; ++a) {
            double d = pos[3 * p + a] - corner[a];
            d -= floor(d);
            if (d > n[a] * h + 2.0 * h) d -= 1.0;
            const double u = d / h;
            if (scheme == 1) {
                const double f = floor(u - 0.5);
                const double t = (u - 0.5) - f;
                c[a][0] = (int)f;
                c[a][1] = (int)f + 1;
                w[a][0] = 1.0 - t;
                w[a][1] = t;
            } else {
                const double f = floor(u);
                const double dd = u - (f + 0.5);
                for (int q = 0; q < 3; ++q) c[a][q] = (int)f + q - 1;
                w[a][0] = 0.5 * (0.5 - dd) * (0.5 - dd);
                w[a][1] = 0.75 - dd * dd;
                w[a][2] = 0.5 * (0.5 + dd) * (0.5 + dd);
            }
        }
        for (int qz = 0; qz < m; ++qz)
            for (int qy = 0; qy < m; ++qy)
                for (int qx = 0; qx < m; ++qx) {
                    const int i = c[0][qx], j = c[1][qy], k = c[2][qz];
                    if (i < 0 || i >= n[0] || j < 0 || j >= n[1] || k < 0 || k >= n[2]) continue;
                    delta[((long)k * n[1] + j) * n[0] + i] += w[0][qx] * w[1][qy] * w[2][qz];
                }
    }
    for (long e = 0; e < N; ++e) delta[e] = delta[e] / mean_count - 1.0;
    return 0;
}
