// Host side of the gfx950 multigrid library: plans, level hierarchies, the
// FAS V-cycle (Li, Zhao & Koyama, Sec. III.C), the convergence loop, hipGraph
// replay of a cycle, and the extern "C" entry points declared in vmg.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/vmg.h"
#include "vmg_internal.h"
#include <rocprofiler-sdk-roctx/roctx.h>

#include "vmg_plan.h"

namespace vmg {

thread_local std::string g_err;

vmg_status fail(vmg_status st, const std::string& msg) {
    g_err = msg;
    return st;
}

#define CKH(expr)                                                                        \
    do {                                                                                 \
        hipError_t _e = (expr);                                                          \
        if (_e != hipSuccess)                                                            \
            return fail(VMG_EHIP, std::string(#expr) + ": " + hipGetErrorString(_e));    \
    } while (0)

static Geom make_geom(int n0, int n1, int n2, bool dirichlet, double h) {
    Geom g;
    g.n0 = n0; g.n1 = n1; g.n2 = n2;
    g.dir = dirichlet ? 1 : 0;
    g.h = h;
    g.base = 0;
    g.ncell = (int64_t)n0 * n1 * n2;
    if (dirichlet) {
        g.sy = n0 + 2;
        g.sz = g.sy * (n1 + 2);
        g.off0 = 1 + g.sy + g.sz;
        g.nstore = g.sz * (n2 + 2);
    } else {
        g.sy = n0;
        g.sz = (int64_t)n0 * n1;
        g.off0 = 0;
        g.nstore = g.ncell;
    }
    return g;
}

static bool can_coarsen(const Geom& g) {
    const int minc = g.dir ? 2 : 4;
    const int n[3] = {g.n0, g.n1, g.n2};
    for (int d = 0; d < 3; ++d)
        if ((n[d] & 1) || n[d] / 2 < minc) return false;
    return true;
}

Coef make_coef(double alpha, double kappa) {
    Coef c;
    c.alpha = alpha;
    c.kappa = kappa;
    c.c8 = 8.0 * alpha / 3.0;
    c.vertex = alpha != 0.0 ? -3.0 / (4.0 * alpha) : 0.0;
    c.sqrt_form = std::fabs(alpha) >= 1e-2 ? 1 : 0;
    return c;
}

static vmg_status dalloc(Plan* P, void** p, size_t bytes) {
    if (hipMalloc(p, bytes) != hipSuccess) return fail(VMG_ENOMEM, "hipMalloc failed");
    P->allocs.push_back(*p);
    return VMG_OK;
}

// ---------------------------------------------------------------------------
vmg_status build_plan(Plan* P, const vmg_grid* grids, int n_grids, const vmg_params* p,
                      hipStream_t stream) {
    if (!stream) {
        // stream capture is not possible on the legacy null stream: use a blocking
        // stream of our own (default priority; it synchronises with the null stream)
        CKH(hipStreamCreate(&P->own_stream));
        stream = P->own_stream;
    }
    P->stream = stream;
    P->params = *p;
    P->coef = make_coef(p->alpha, p->kappa);
    P->nu1 = p->nu1;
    P->nu2 = p->nu2;
    if (P->nu1 == 0 && P->nu2 == 0) { P->nu1 = 2; P->nu2 = 2; }
    P->inner = p->inner_cycles > 0 ? p->inner_cycles : 2;
    P->ncoarse = 8;
    P->cfg.ty = 8;
    P->cfg.zc = 16;
    P->periodic = grids[0].bc == VMG_PERIODIC;
    int64_t max_cells = 1;
    for (int gi = 0; gi < n_grids; ++gi) {
        const vmg_grid& d = grids[gi];
        GridState G;
        G.desc = d;
        Geom g = make_geom(d.n[0], d.n[1], d.n[2], d.bc == VMG_DIRICHLET, d.h);
        for (;;) {
            LevelBuf L;
            L.g = g;
            G.lev.push_back(L);
            if (!can_coarsen(g) || G.lev.size() >= 24) break;
            g = make_geom(g.n0 / 2, g.n1 / 2, g.n2 / 2, g.dir == 1, g.h * 2.0);
        }
        const Geom& gc = G.lev.back().g;
        if (gc.n0 > 8 || gc.n1 > 8 || gc.n2 > 8)
            return fail(VMG_EINVAL, "grid " + std::to_string(gi) + " does not coarsen to <= 8 cells per side");
        max_cells = std::max<int64_t>(max_cells, G.lev[0].g.ncell);
        P->grids.push_back(G);
    }
    P->mixed = p->prec == VMG_MIXED;
    P->batched = !P->periodic;
    vmg_status st;
    if (P->batched) {
        if ((st = build_batch(P)) != VMG_OK) return st;
    } else {
        for (auto& G : P->grids) {
            for (size_t l = 0; l < G.lev.size(); ++l) {
                LevelBuf& L = G.lev[l];
                const size_t bytes = sizeof(double) * (size_t)L.g.nstore;
                if ((st = dalloc(P, (void**)&L.phi[0], bytes)) != VMG_OK) return st;
                if ((st = dalloc(P, (void**)&L.phi[1], bytes)) != VMG_OK) return st;
                if ((st = dalloc(P, (void**)&L.delta, bytes)) != VMG_OK) return st;
                if ((st = dalloc(P, (void**)&L.f, bytes)) != VMG_OK) return st;
                if (l > 0) {
                    if ((st = dalloc(P, (void**)&L.phiold, bytes)) != VMG_OK) return st;
                    if ((st = dalloc(P, (void**)&L.rd, bytes)) != VMG_OK) return st;
                }
                if ((st = dalloc(P, (void**)&L.sc, sizeof(LevelScalars))) != VMG_OK) return st;
                CKH(launch_fill(L.phi[0], L.g.nstore, 0.0, stream));
                CKH(launch_fill(L.phi[1], L.g.nstore, 0.0, stream));
                CKH(launch_fill(L.f, L.g.nstore, 0.0, stream));
                CKH(launch_fill(L.delta, L.g.nstore, 0.0, stream));
                if (l > 0) {
                    CKH(launch_fill(L.phiold, L.g.nstore, 0.0, stream));
                    CKH(launch_fill(L.rd, L.g.nstore, 0.0, stream));
                }
                CKH(launch_fill((double*)L.sc, sizeof(LevelScalars) / sizeof(double), 0.0, stream));
            }
        }
        if (P->mixed && (st = alloc_mixed(P)) != VMG_OK) return st;
    }
    for (auto& G : P->grids) {
        if ((st = dalloc(P, (void**)&G.norm_dev, sizeof(NormOut))) != VMG_OK) return st;
        CKH(launch_fill((double*)G.norm_dev, sizeof(NormOut) / sizeof(double), 0.0, stream));
    }
    int64_t nb = partial_blocks_for(max_cells);
    for (auto& G : P->grids)
        for (auto& L : G.lev) nb = std::max<int64_t>(nb, resid_blocks(L.g));
    nb = std::max<int64_t>(nb, batch_partials_needed(P));
    if ((st = dalloc(P, (void**)&P->partials, 2 * sizeof(double) * R_NSLOT * (size_t)nb)) != VMG_OK) return st;
    P->partials_b = P->partials + R_NSLOT * (size_t)nb;
    if (hipHostMalloc((void**)&P->host_norm, sizeof(NormOut) * P->grids.size(), hipHostMallocDefault) !=
        hipSuccess)
        return fail(VMG_ENOMEM, "hipHostMalloc failed");
    CKH(hipStreamSynchronize(stream));
    if (p->flags & VMG_AUTOTUNE) {
        if ((st = autotune(P)) != VMG_OK) return st;
        CKH(hipStreamSynchronize(stream));
    }
    return VMG_OK;
}

static void release_graphs(Plan* P);

void destroy_plan(Plan* P) {
    release_graphs(P);
    for (hipEvent_t ev : P->tev) (void)hipEventDestroy(ev);
    for (hipEvent_t ev : P->lev_ev) (void)hipEventDestroy(ev);
    for (void* a : P->allocs) (void)hipFree(a);
    if (P->host_norm) (void)hipHostFree(P->host_norm);
    if (P->own_stream) (void)hipStreamDestroy(P->own_stream);
}

// ---------------------------------------------------------------------------
// one V-cycle on one grid
// ---------------------------------------------------------------------------
static const double* level_f(const Plan* P, const GridState& G, int l) {
    if (l > 0) return G.lev[l].f;
    return P->has_source ? G.lev[0].f : nullptr;
}

hipError_t sweep_mark(Plan* P, bool begin, int launches) {
    if (!P->time_sweeps || !P->timing_active || launches <= 0 || P->tev_used >= (int)P->tev.size() / 2)
        return hipSuccess;
    if (begin) return hipEventRecord(P->tev[2 * P->tev_used], P->stream);
    P->tev_count[P->tev_used] = launches;
    return hipEventRecord(P->tev[2 * P->tev_used++ + 1], P->stream);
}

// accumulate the durations of the first n recorded runs of sweep launches
// (after the stream has finished them)
static hipError_t collect_sweeps(Plan* P, int n) {
    for (int i = 0; i < n; ++i) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, P->tev[2 * i], P->tev[2 * i + 1]);
        if (e != hipSuccess) return e;
        P->sweep_us += 1e3 * ms;
        P->sweep_n += P->tev_count[i];
    }
    P->tev_used = 0;
    return hipSuccess;
}

// Per-level timing: event pairs tagged with the level, and a ROCTX range per piece.
hipError_t level_mark(Plan* P, int l, bool begin) {
    if (!P->time_levels || !P->timing_active) return hipSuccess;
    if (begin) {
        if (P->lev_used >= (int)P->lev_tag.size()) return hipSuccess;   // pool full: piece not timed
        static const char* names[] = {"vmg level 0", "vmg level 1", "vmg level 2", "vmg level 3",
                                      "vmg level 4", "vmg level 5", "vmg level 6", "vmg level 7",
                                      "vmg level 8", "vmg level 9", "vmg level 10+"};
        roctxRangePushA(names[l < 10 ? l : 10]);
        P->lev_tag[P->lev_used] = -1 - l;   // open
        return hipEventRecord(P->lev_ev[2 * P->lev_used], P->stream);
    }
    if (P->lev_used >= (int)P->lev_tag.size() || P->lev_tag[P->lev_used] != -1 - l) return hipSuccess;
    roctxRangePop();
    P->lev_tag[P->lev_used] = l;
    return hipEventRecord(P->lev_ev[2 * P->lev_used++ + 1], P->stream);
}

// accumulate the recorded pieces (after the stream has finished them)
static hipError_t collect_levels(Plan* P) {
    for (int i = 0; i < P->lev_used; ++i) {
        float ms = 0.0f;
        hipError_t e = hipEventElapsedTime(&ms, P->lev_ev[2 * i], P->lev_ev[2 * i + 1]);
        if (e != hipSuccess) return e;
        const int l = P->lev_tag[i];
        if (l >= 0 && l < (int)P->level_us.size()) P->level_us[l] += 1e3 * ms;
    }
    P->lev_used = 0;
    return hipSuccess;
}

// `count` sweeps of level l, the first from phi + the prolonged coarse correction
// when `pro` is given: one launch per sweep, or per two on the brick schedule
static hipError_t smooth_level_n(Plan* P, GridState& G, int l, int count, const ProlongIn* pro = nullptr) {
    LevelBuf& L = G.lev[l];
    const SmoothCfg cfg = level_schedule(P, l, L.g);
    const int per = cfg.pipe == PIPE_BRICK ? 2 : 1;
    for (int s = 0; s < count;) {
        const int n = std::min(per, count - s);
        hipError_t e = launch_smooth(L.g, P->coef, L.phi[L.cur], L.phi[L.cur ^ 1], L.delta, level_f(P, G, l), L.sc,
                                     cfg, P->stream, s == 0 ? pro : nullptr, n);
        L.cur ^= 1;
        P->cell_updates += n * L.g.ncell;
        if (l == 0) P->finest_sweeps += n;
        if (e != hipSuccess) return e;
        s += n;
    }
    return hipSuccess;
}

static hipError_t smooth_level(Plan* P, GridState& G, int l, const ProlongIn* pro = nullptr) {
    return smooth_level_n(P, G, l, 1, pro);
}

hipError_t smooth_level_public(Plan* P, GridState& G, int l, int count) { return smooth_level_n(P, G, l, count); }

bool fold_prolong_here(const Plan* P, const Geom& g, const Geom& gc, const SmoothCfg& cfg) {
    if (!P->fold_prolong) return false;
    if (cfg.pipe == PIPE_BRICK) return can_fold_prolong(g, gc, 2);
    const int zc = cfg.zc > 0 ? cfg.zc : 16;
    return can_fold_prolong(g, gc, zc) && fold_prolong_pays(g, zc);
}

// The finest level runs the plan's schedule; a coarser level its tuned one, else
// the plan's schedule shortened by level_cfg.
SmoothCfg level_schedule(const Plan* P, int l, const Geom& g) {
    if (l == 0) return P->cfg;
    if ((int)P->lcfg.size() > l && P->lcfg[l].ty > 0) return P->lcfg[l];
    return level_cfg(g.n0, g.n1, g.n2, P->cfg);
}

// First level (below the finest) at which the periodic coarse tail takes over,
// or -1 when the plan does not use it.
int tail_level(const Plan* P, const GridState& G) {
    if (!P->use_tail || G.lev.empty() || G.lev[0].g.dir) return -1;
    const int last = (int)G.lev.size() - 1;
    for (int l = 1; l <= last; ++l)
        if (G.lev[l].g.ncell <= TAIL_CELLS) return last - l + 1 <= TAIL_LEVELS ? l : -1;
    return -1;
}

static hipError_t tail_cycle(Plan* P, GridState& G, int l) {
    const int last = (int)G.lev.size() - 1;
    TailArgs a;
    a.nlev = last - l + 1;
    for (int q = 0; q < a.nlev; ++q) {
        const LevelBuf& T = G.lev[l + q];
        a.n[q][0] = T.g.n0; a.n[q][1] = T.g.n1; a.n[q][2] = T.g.n2;
        a.h[q] = T.g.h;
        a.delta[q] = T.delta;
        P->cell_updates += (int64_t)(q == a.nlev - 1 ? P->ncoarse : pre_sweeps(P, l + q) + post_sweeps(P, l + q)) *
                           T.g.ncell;
    }
    LevelBuf& L = G.lev[l];
    a.phi = L.phi[L.cur];
    a.f = level_f(P, G, l);
    a.sc = L.sc;
    a.c = P->coef;
    a.nu1 = pre_sweeps(P, l); a.nu2 = post_sweeps(P, l); a.ncoarse = P->ncoarse;
    return launch_tail(a, P->stream);
}

static hipError_t vcycle(Plan* P, GridState& G, int l);

// A V-cycle on level l < last in two parts.  The head pre-smooths, then one
// pass computes the residual and restricts phi and d to level l+1, and a second
// forms the coarse right-hand side f^H = L^H(R phi) - R d (Sec. III.C); one
// two-block launch closes both passes' reductions: the new cbar of both levels
// and, with `norm`, the RMS of the pre-smoothed state's residual and of its
// truncation-error estimate tau^h = L^H(R phi) - R L^h(phi) (Sec. III.C; only
// the finest level asks for them).  The tail runs the coarse cycle, prolongs
// and post-smooths.
static hipError_t vcycle_head(Plan* P, GridState& G, int l, NormOut* norm) {
    LevelBuf& L = G.lev[l];
    hipError_t e;
    if ((e = level_mark(P, l, true)) != hipSuccess) return e;
    const int nu1 = pre_sweeps(P, l);
    if (l == 0 && (e = sweep_mark(P, true, nu1)) != hipSuccess) return e;
    if ((e = smooth_level_n(P, G, l, nu1)) != hipSuccess) return e;
    if (l == 0 && (e = sweep_mark(P, false, nu1)) != hipSuccess) return e;
    LevelBuf& C = G.lev[l + 1];
    C.cur = 0;
    int nb = 0, nbc = 0;
    if ((e = launch_residual_restrict(L.g, C.g, P->coef, L.phi[L.cur], L.delta, level_f(P, G, l), L.sc,
                                      C.phi[0], C.phiold, C.rd, P->partials, &nb, P->stream)) != hipSuccess)
        return e;
    if ((e = launch_fas_rhs(C.g, P->coef, C.phi[0], C.delta, C.rd, C.f, P->partials_b, &nbc, P->stream,
                            norm ? level_f(P, G, l) : nullptr, &L.g)) != hipSuccess)
        return e;
    // with Dirichlet faces there is no cbar: only the norms need finalizing
    const int periodic = L.g.dir ? 0 : 1;
    if (!periodic && !norm) return level_mark(P, l, false);
    if ((e = launch_finalize_pair(FinJob{P->partials, nb, periodic, 0, L.g.ncell, L.sc, norm, nullptr},
                                  FinJob{P->partials_b, nbc, periodic, 1, C.g.ncell, C.sc, norm, nullptr},
                                  P->stream)) != hipSuccess)
        return e;
    return level_mark(P, l, false);
}

// phi^h += P(phi^H - phi^H_old), then nu2 sweeps of level l: on periodic grids
// the prolongation is folded into the first sweep where that pays (on the
// finest level that sweep is not timed with the plain ones)
hipError_t post_smooth(Plan* P, GridState& G, int l, int nu2) {
    LevelBuf& L = G.lev[l];
    LevelBuf& C = G.lev[l + 1];
    hipError_t e;
    const int s0 = nu2 > 0 && fold_prolong_here(P, L.g, C.g, level_schedule(P, l, L.g)) ? 1 : 0;
    const ProlongIn pro{C.g, C.phi[C.cur], C.phiold};
    if (!s0 && (e = launch_prolong(L.g, C.g, L.phi[L.cur], C.phi[C.cur], C.phiold, P->stream)) != hipSuccess)
        return e;
    if (l > 0) return smooth_level_n(P, G, l, nu2, s0 ? &pro : nullptr);
    if (s0 && (e = smooth_level(P, G, l, &pro)) != hipSuccess) return e;
    if ((e = sweep_mark(P, true, nu2 - s0)) != hipSuccess) return e;
    if ((e = smooth_level_n(P, G, l, nu2 - s0)) != hipSuccess) return e;
    return sweep_mark(P, false, nu2 - s0);
}

static hipError_t vcycle_tail(Plan* P, GridState& G, int l) {
    hipError_t e;
    if ((e = vcycle(P, G, l + 1)) != hipSuccess) return e;
    if ((e = level_mark(P, l, true)) != hipSuccess) return e;
    if ((e = post_smooth(P, G, l, post_sweeps(P, l))) != hipSuccess) return e;
    return level_mark(P, l, false);
}

static hipError_t vcycle(Plan* P, GridState& G, int l) {
    LevelBuf& L = G.lev[l];
    const int last = (int)G.lev.size() - 1;
    hipError_t e;
    if (l > 0 && l == tail_level(P, G)) {
        if ((e = level_mark(P, l, true)) != hipSuccess || (e = tail_cycle(P, G, l)) != hipSuccess) return e;
        return level_mark(P, l, false);
    }
    if (l == last) {
        if ((e = level_mark(P, l, true)) != hipSuccess) return e;
        e = launch_coarse_solve(L.g, P->coef, L.phi[L.cur], L.delta, level_f(P, G, l), L.sc,
                                P->ncoarse, P->stream);
        P->cell_updates += (int64_t)P->ncoarse * L.g.ncell;
        if (e != hipSuccess) return e;
        return level_mark(P, l, false);
    }
    if ((e = vcycle_head(P, G, l, nullptr)) != hipSuccess) return e;
    return vcycle_tail(P, G, l);
}

static hipError_t norm_pass(Plan* P, GridState& G) {
    LevelBuf& L = G.lev[0];
    int nb = 0;
    hipError_t e = launch_residual_norm(L.g, P->coef, L.phi[L.cur], L.delta, level_f(P, G, 0), L.sc,
                                        nullptr, P->partials, &nb, P->stream);
    if (e != hipSuccess) return e;
    return launch_finalize(P->partials, nb, L.g.ncell, L.g.dir ? 0 : 1, 0, L.sc, G.norm_dev, P->stream);
}

// FP64 cycles on a grid with coarser levels are run shifted by one head: the
// convergence test reads the residual of the pre-smoothed state, which the
// finest residual-and-restriction pass computes anyway, so no separate norm
// pass is needed.  The solve runs one head, then units (tail of cycle k, head
// of cycle k+1) until that residual meets the tolerance; the result is the
// pre-smoothed state whose residual was measured.
constexpr int DIVERGE_GRACE = 4;   // iterations before the 10x divergence rule applies

static bool shifted_cycles(const Plan* P) {
    if (P->mixed || P->batched) return false;
    for (const auto& G : P->grids)
        if (G.lev.size() < 2) return false;
    return true;
}

static hipError_t norms_to_host_fp64(Plan* P) {
    for (size_t gi = 0; gi < P->grids.size(); ++gi) {
        hipError_t e = hipMemcpyAsync(&P->host_norm[gi], P->grids[gi].norm_dev, sizeof(NormOut),
                                      hipMemcpyDeviceToHost, P->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

// The first head of a shifted solve (pre-smoothing and the residual of its result).
static hipError_t enqueue_first_head(Plan* P) {
    hipError_t e;
    for (auto& G : P->grids)
        if ((e = vcycle_head(P, G, 0, G.norm_dev)) != hipSuccess) return e;
    return norms_to_host_fp64(P);
}

// Enqueue one cycle for every grid + norms + the copy of the norms to the host:
// a full cycle and a norm pass, or (shifted) the tail of one cycle and the head
// of the next.
static hipError_t enqueue_cycle(Plan* P) {
    hipError_t e;
    const bool shifted = shifted_cycles(P);
    for (auto& G : P->grids) {
        if (shifted) {
            if ((e = vcycle_tail(P, G, 0)) != hipSuccess) return e;
            if ((e = vcycle_head(P, G, 0, G.norm_dev)) != hipSuccess) return e;
        } else {
            if ((e = vcycle(P, G, 0)) != hipSuccess) return e;
            if ((e = norm_pass(P, G)) != hipSuccess) return e;
        }
    }
    return norms_to_host_fp64(P);
}

static hipError_t enqueue_iteration(Plan* P) {
    if (P->batched) return batch_enqueue_iteration(P);
    return P->mixed ? enqueue_outer(P) : enqueue_cycle(P);
}

static int finest_parity(const Plan* P) { return P->batched ? batch_parity(P) : P->grids[0].lev[0].cur; }

static void release_graphs(Plan* P) {
    for (int src = 0; src < 2; ++src)
        for (int q = 0; q < 2; ++q)
            if (P->graph_ok[src][q]) {
                (void)hipGraphExecDestroy(P->graph[src][q]);
                P->graph_ok[src][q] = false;
            }
}

// Record one iteration (enqueue_iteration) as a hipGraph for the given source
// flag and finest-level parity.  Capture only records work, so every piece of
// host-side state that enqueueing advances is restored afterwards; the
// iteration's cell-update counts are kept for the replays.
static vmg_status capture_graph(Plan* P, int src, int parity) {
    std::vector<int> saved;
    for (auto& G : P->grids) saved.push_back(G.lev[0].cur);
    const int saved_b = finest_parity(P);
    const bool saved_src = P->has_source;
    P->has_source = src != 0;
    if (P->batched) {
        if (batch_parity(P) != parity) batch_flip_parity(P);
    } else {
        for (auto& G : P->grids) G.lev[0].cur = parity;
    }
    const int64_t cu = P->cell_updates, fs = P->finest_sweeps;
    hipGraph_t graph;
    P->tev_used = 0;
    P->timing_active = true;
    hipError_t e0 = hipStreamBeginCapture(P->stream, hipStreamCaptureModeThreadLocal);
    hipError_t e = e0 == hipSuccess ? enqueue_iteration(P) : e0;
    hipError_t e2 = e0 == hipSuccess ? hipStreamEndCapture(P->stream, &graph) : e0;
    P->timing_active = false;
    P->graph_tev[src][parity] = P->tev_used;
    P->tev_used = 0;
    P->graph_updates[src][parity] = P->cell_updates - cu;
    P->graph_finest[src][parity] = P->finest_sweeps - fs;
    // where the iteration leaves the finest phi: each launch on it flips the
    // ping-pong buffers (the mixed path's update pass once per iteration)
    P->graph_flip[src][parity] = finest_parity(P) != parity;
    P->cell_updates = cu;
    P->finest_sweeps = fs;
    for (size_t gi = 0; gi < P->grids.size(); ++gi) P->grids[gi].lev[0].cur = saved[gi];
    if (P->batched && batch_parity(P) != saved_b) batch_flip_parity(P);
    P->has_source = saved_src;
    if (e != hipSuccess) return fail(VMG_EHIP, std::string("graph capture: ") + hipGetErrorString(e));
    CKH(e2);
    hipError_t ei = hipGraphInstantiate(&P->graph[src][parity], graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    CKH(ei);
    P->graph_ok[src][parity] = true;
    return VMG_OK;
}

// With VMG_GRAPH, record the iteration for both source flags and both
// finest-level parities (so a solve replays without instantiating anything);
// called when a plan is created and again when its schedule changes.
vmg_status capture_graphs(Plan* P) {
    release_graphs(P);
    // event-record nodes of a graph carry no timestamps on this runtime, so a
    // plan that times its sweeps issues its iterations directly
    if (!(P->params.flags & VMG_GRAPH) || P->time_sweeps || P->time_levels) return VMG_OK;
    for (int src = 0; src < 2; ++src)
        for (int q = 0; q < 2; ++q) {
            vmg_status st = capture_graph(P, src, q);
            if (st != VMG_OK) return st;
        }
    return VMG_OK;
}

void get_cycle(const Plan* P, vmg_cycle* c) {
    c->nu1 = P->nu1;
    c->nu2 = P->nu2;
    c->inner_cycles = P->mixed ? P->inner : 0;
    c->coarse_sweeps = P->ncoarse;
    c->coarse_tail = P->periodic && P->use_tail ? 1 : 0;
    c->batch_blocks = P->batched ? P->batch_blocks : 0;
    c->coarse_nu1 = P->nu1c;
    c->coarse_nu2 = P->nu2c;
}

vmg_status set_cycle(Plan* P, const vmg_cycle* c) {
    if (c->nu1 < 0 || c->nu1 > 8 || c->nu2 < 0 || c->nu2 > 8 || c->nu1 + c->nu2 < 1)
        return fail(VMG_EINVAL, "cycle: nu1, nu2 in [0, 8] with nu1 + nu2 >= 1");
    if (P->mixed ? (c->inner_cycles < 1 || c->inner_cycles > 8) : c->inner_cycles != 0)
        return fail(VMG_EINVAL, "cycle: inner_cycles in [1, 8] for mixed plans, 0 for FP64 plans");
    if (c->coarse_sweeps < 1 || c->coarse_sweeps > 64) return fail(VMG_EINVAL, "cycle: coarse_sweeps in [1, 64]");
    if ((c->coarse_tail != 0 && c->coarse_tail != 1) || (!P->periodic && c->coarse_tail != 0))
        return fail(VMG_EINVAL, "cycle: coarse_tail 0 or 1 (periodic plans), 0 (Dirichlet plans)");
    if (P->batched ? (c->batch_blocks < 64 || c->batch_blocks > 65536) : c->batch_blocks != 0)
        return fail(VMG_EINVAL, "cycle: batch_blocks in [64, 65536] for Dirichlet plans, 0 for periodic plans");
    if (c->coarse_nu1 < 0 || c->coarse_nu1 > 8 || c->coarse_nu2 < 0 || c->coarse_nu2 > 8)
        return fail(VMG_EINVAL, "cycle: coarse_nu1, coarse_nu2 in [0, 8] (both 0: nu1, nu2)");
    P->nu1 = c->nu1;
    P->nu2 = c->nu2;
    P->nu1c = c->coarse_nu1;
    P->nu2c = c->coarse_nu2;
    if (P->mixed) P->inner = c->inner_cycles;
    P->ncoarse = c->coarse_sweeps;
    if (P->periodic) P->use_tail = c->coarse_tail != 0;
    if (P->batched) P->batch_blocks = c->batch_blocks;
    CKH(hipStreamSynchronize(P->stream));
    return capture_graphs(P);
}

static vmg_status run_cycle(Plan* P) {
    const int src = P->has_source ? 1 : 0;
    const int parity = finest_parity(P);
    if (!(P->params.flags & VMG_GRAPH) || !P->graph_ok[src][parity]) {
        CKH(enqueue_iteration(P));
        CKH(hipStreamSynchronize(P->stream));
        if (P->time_sweeps) CKH(collect_sweeps(P, P->tev_used));
        if (P->time_levels) {
            CKH(collect_levels(P));
            ++P->level_cycles;
        }
        return VMG_OK;
    }
    CKH(hipGraphLaunch(P->graph[src][parity], P->stream));
    CKH(hipStreamSynchronize(P->stream));
    if (P->time_sweeps) CKH(collect_sweeps(P, P->graph_tev[src][parity]));
    P->cell_updates += P->graph_updates[src][parity];
    P->finest_sweeps += P->graph_finest[src][parity];
    // the replayed iteration leaves the finest phi where the captured one did
    const bool flip = P->graph_flip[src][parity];
    if (flip) {
        if (P->batched)
            batch_flip_parity(P);
        else
            for (auto& G : P->grids) G.lev[0].cur ^= 1;
    }
    return VMG_OK;
}

// ---------------------------------------------------------------------------
vmg_status solve(Plan* P, const double* delta, const double* ghost, const double* source, double* phi,
                 vmg_result* out) {
    hipStream_t s = P->stream;
    P->timing_active = false;
    P->has_source = source != nullptr;
    P->cell_updates = 0;
    P->finest_sweeps = 0;
    // ---- inputs -> plan buffers ------------------------------------------
    int nb = 0;
    if (P->batched) {
        CKH(batch_check_delta(P, delta));
    } else {
        for (auto& G : P->grids) {
            LevelBuf& L0 = G.lev[0];
            const double* d_in = delta + G.desc.offset;
            CKH(launch_check_finite(d_in, L0.g.ncell, P->partials, &nb, s));
            CKH(launch_finalize(P->partials, nb, L0.g.ncell, 0, 0, L0.sc, G.norm_dev, s));
            CKH(hipMemcpyAsync(&P->host_norm[&G - &P->grids[0]], G.norm_dev, sizeof(NormOut),
                               hipMemcpyDeviceToHost, s));
        }
    }
    CKH(hipStreamSynchronize(s));
    for (size_t gi = 0; gi < P->grids.size(); ++gi)
        if (P->host_norm[gi].n_nonfinite > 0)
            return fail(VMG_ENONFINITE, "non-finite values in delta of grid " + std::to_string(gi));
    if (P->batched) {
        CKH(batch_setup(P, delta, ghost, source, phi));
    } else {
    for (auto& G : P->grids) {
        LevelBuf& L0 = G.lev[0];
        L0.cur = 0;
        CKH(launch_copy_in(L0.g, delta + G.desc.offset, L0.delta, s));
        CKH(launch_copy_in(L0.g, phi + G.desc.offset, L0.phi[0], s));
        if (source) CKH(launch_copy_in(L0.g, source + G.desc.offset, L0.f, s));
        if (L0.g.dir) {
            CKH(launch_ghost_in(L0.g, ghost + G.desc.ghost_offset, L0.phi[0], s));
            CKH(launch_ghost_in(L0.g, ghost + G.desc.ghost_offset, L0.phi[1], s));
        }
        for (size_t l = 1; l < G.lev.size(); ++l) {
            LevelBuf& F = G.lev[l - 1];
            LevelBuf& C = G.lev[l];
            CKH(launch_restrict_plain(F.g, C.g, F.delta, C.delta, s));
            if (C.g.dir) {
                CKH(launch_restrict_ghosts(F.g, C.g, F.phi[0], C.phi[0], s));
                CKH(launch_restrict_ghosts(F.g, C.g, F.phi[0], C.phi[1], s));
                CKH(launch_restrict_ghosts(F.g, C.g, F.phi[0], C.phiold, s));
            }
        }
        for (auto& L : G.lev) CKH(launch_fill((double*)L.sc, sizeof(LevelScalars) / sizeof(double), 0.0, s));
        if (!P->mixed) CKH(norm_pass(P, G));
    }
    if (P->mixed) {
        CKH(mixed_prepare(P));
        CKH(mixed_initial_pass(P));
    } else {
        for (size_t gi = 0; gi < P->grids.size(); ++gi)
            CKH(hipMemcpyAsync(&P->host_norm[gi], P->grids[gi].norm_dev, sizeof(NormOut),
                               hipMemcpyDeviceToHost, s));
    }
    }
    CKH(hipStreamSynchronize(s));
    const int ng = (int)P->grids.size();
    std::vector<double> rms0(ng), best(ng);
    auto record = [&]() {
        for (int gi = 0; gi < ng; ++gi) {
            const NormOut& no = P->host_norm[gi];
            P->history[gi].push_back(vmg_history{no.rms, no.cbar, no.n_guard, no.tau_rms});
        }
    };
    P->history.assign(ng, std::vector<vmg_history>());
    for (int gi = 0; gi < ng; ++gi) {
        rms0[gi] = P->host_norm[gi].rms;
        best[gi] = rms0[gi];
        if (!(P->host_norm[gi].n_nonfinite == 0) || !std::isfinite(rms0[gi]))
            return fail(VMG_ENONFINITE, "non-finite initial residual in grid " + std::to_string(gi));
    }
    // ---- cycles ------------------------------------------------------------
    int cycles = 0;
    std::vector<int> worse(ng, 0);   // consecutive iterations more than 10x above the best RMS
    vmg_status status = VMG_OK;
    // tau_rms is written by the heads of shifted cycles only; 0 before the first
    const double tf = P->params.tau_factor;
    for (int gi = 0; gi < ng; ++gi) P->host_norm[gi].tau_rms = 0.0;
    record();
    auto converged = [&]() {
        for (int gi = 0; gi < ng; ++gi) {
            const NormOut& no = P->host_norm[gi];
            const bool by_tol = no.rms <= P->params.tol;
            const bool by_tau = tf > 0.0 && no.tau_rms > 0.0 && no.rms <= tf * no.tau_rms;
            if (!(by_tol || by_tau)) return false;
        }
        return true;
    };
    P->timing_active = true;
    P->tev_used = 0;
    if (shifted_cycles(P) && !converged()) {
        CKH(enqueue_first_head(P));
        CKH(hipStreamSynchronize(s));
        if (P->time_sweeps) CKH(collect_sweeps(P, P->tev_used));
        if (P->time_levels) CKH(collect_levels(P));
    }
    while (!converged()) {
        if (cycles >= P->params.max_cycles) {
            status = VMG_ENOCONV;
            break;
        }
        roctxRangePushA("vmg iteration");
        vmg_status st = run_cycle(P);
        roctxRangePop();
        if (st != VMG_OK) return st;
        ++cycles;
        record();
        // divergence: a non-finite residual, one 1e4 times above the best so far, or
        // three iterations in a row 10 times above it once the first few iterations
        // (whose nonlinear start phase may raise the residual) are past
        bool bad = false;
        for (int gi = 0; gi < ng; ++gi) {
            const NormOut& no = P->host_norm[gi];
            const double b = std::max(best[gi], 1e-300);
            worse[gi] = (cycles > DIVERGE_GRACE && no.rms > 10.0 * b) ? worse[gi] + 1 : 0;
            if (no.n_nonfinite > 0 || !std::isfinite(no.rms) || no.rms > 1e4 * b || worse[gi] >= 3) bad = true;
            best[gi] = std::min(best[gi], no.rms);
        }
        if (bad) {
            status = VMG_ENONFINITE;
            g_err = "residual became non-finite or diverged";
            break;
        }
    }
    P->timing_active = false;
    // ---- outputs -------------------------------------------------------------
    if (P->batched) CKH(batch_outputs(P, phi));
    for (int gi = 0; gi < ng; ++gi) {
        GridState& G = P->grids[gi];
        LevelBuf& L0 = G.lev[0];
        if (!P->batched) {
            if (!L0.g.dir) CKH(launch_gauge(L0.g, L0.phi[L0.cur], G.norm_dev, s));
            CKH(launch_copy_out(L0.g, L0.phi[L0.cur], phi + G.desc.offset, s));
        }
        if (out) {
            out[gi].rms0 = rms0[gi];
            out[gi].rms = P->host_norm[gi].rms;
            out[gi].compat_c = P->host_norm[gi].cbar;
            out[gi].cycles = cycles;
            out[gi].inner_cycles = P->mixed ? cycles * P->inner : 0;
            out[gi].n_guarded = (int64_t)P->host_norm[gi].n_guard;
            out[gi].tau_rms = tf > 0.0 ? P->host_norm[gi].tau_rms : 0.0;
        }
    }
    CKH(hipStreamSynchronize(s));
    P->solved = true;
    if (status == VMG_ENOCONV) g_err = "max_cycles reached before the tolerance";
    return status;
}

}  // namespace vmg

// ===========================================================================
// C ABI
// ===========================================================================
using namespace vmg;

extern "C" {

const char* vmg_last_error(void) { return g_err.c_str(); }

int64_t vmg_ghost_count(const int32_t n[3]) {
    if (!n) return 0;
    return ghost_count(n[0], n[1], n[2]);
}

vmg_status vmg_plan_create(vmg_plan** plan, const vmg_grid* grids, int32_t n_grids, const vmg_params* p,
                           hipStream_t stream) {
    g_err.clear();
    if (!plan || !grids || !p || n_grids < 1) return fail(VMG_EINVAL, "null argument or n_grids < 1");
    *plan = nullptr;
    if (!(p->tol > 0.0) || p->max_cycles < 1 || (p->prec != VMG_FP64 && p->prec != VMG_MIXED) ||
        p->nu1 < 0 || p->nu2 < 0 || p->inner_cycles < 0 || (p->prec == VMG_FP64 && p->inner_cycles != 0) ||
        !std::isfinite(p->alpha) || !std::isfinite(p->kappa) || !(p->tau_factor >= 0.0) ||
        !std::isfinite(p->tau_factor))
        return fail(VMG_EINVAL, "invalid parameters (tol > 0, max_cycles >= 1, prec, nu1/nu2 >= 0, finite alpha/kappa, "
                                "tau_factor >= 0)");
    const int bc0 = grids[0].bc;
    for (int i = 0; i < n_grids; ++i) {
        const vmg_grid& g = grids[i];
        if (g.bc != VMG_PERIODIC && g.bc != VMG_DIRICHLET) return fail(VMG_EINVAL, "unknown bc");
        if (g.bc != bc0) return fail(VMG_EINVAL, "a plan holds one periodic grid or Dirichlet grids only");
        const int minn = g.bc == VMG_PERIODIC ? 4 : 2;
        if (g.n[0] < minn || g.n[1] < minn || g.n[2] < minn)
            return fail(VMG_EINVAL, "grid too small (periodic >= 4, Dirichlet >= 2 cells per side)");
        if (!(g.h > 0.0) || !std::isfinite(g.h)) return fail(VMG_EINVAL, "h must be > 0");
        if (g.offset < 0 || g.ghost_offset < 0) return fail(VMG_EINVAL, "negative offset");
    }
    if (bc0 == VMG_PERIODIC && n_grids != 1) return fail(VMG_EINVAL, "a periodic plan holds exactly one grid");
    if (p->tau_factor > 0.0)
        for (int i = 0; i < n_grids; ++i) {
            const vmg_grid& g = grids[i];
            if (!can_coarsen(make_geom(g.n[0], g.n[1], g.n[2], g.bc == VMG_DIRICHLET, g.h)))
                return fail(VMG_EINVAL, "tau_factor needs grids with a coarser level (tau^h lives on it); grid " +
                                            std::to_string(i) + " has none");
        }
    Plan* P = new (std::nothrow) Plan();
    if (!P) return fail(VMG_ENOMEM, "host allocation failed");
    vmg_status st = build_plan(P, grids, n_grids, p, stream);
    if (st == VMG_OK && (p->flags & VMG_AUTOTUNE)) {
        // a cycle schedule vmg_plan_tune_cycle cached for this plan's key; the
        // caller's explicit nu1/nu2 and inner_cycles take precedence
        vmg_cycle c;
        if (cached_cycle(P, &c)) {
            if (p->nu1 != 0 || p->nu2 != 0) {
                c.nu1 = P->nu1;
                c.nu2 = P->nu2;
                c.coarse_nu1 = c.coarse_nu2 = 0;
            }
            if (p->inner_cycles != 0) c.inner_cycles = P->inner;
            if (!P->mixed) c.inner_cycles = 0;
            if (!P->periodic) c.coarse_tail = 0;
            if (!P->batched) c.batch_blocks = 0;
            else if (c.batch_blocks == 0) c.batch_blocks = P->batch_blocks;
            st = set_cycle(P, &c);
        }
    }
    if (st == VMG_OK) st = capture_graphs(P);
    if (st != VMG_OK) {
        std::string msg = g_err;
        destroy_plan(P);
        delete P;
        g_err = msg;
        return st;
    }
    *plan = reinterpret_cast<vmg_plan*>(P);
    return VMG_OK;
}

vmg_status vmg_plan_destroy(vmg_plan* plan) {
    if (!plan) return VMG_OK;
    Plan* P = reinterpret_cast<Plan*>(plan);
    (void)hipStreamSynchronize(P->stream);
    destroy_plan(P);
    delete P;
    return VMG_OK;
}

vmg_status vmg_solve(vmg_plan* plan, const double* delta, const double* ghost, const double* source,
                     double* phi, vmg_result* out) {
    g_err.clear();
    if (!plan || !delta || !phi) return fail(VMG_EINVAL, "null plan, delta or phi");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (!P->periodic && !ghost) return fail(VMG_EINVAL, "Dirichlet grids need ghost values");
    roctxRangePushA("vmg_solve");
    const vmg_status st = solve(P, delta, ghost, source, phi, out);
    roctxRangePop();
    return st;
}

vmg_status vmg_solve_periodic(const double* delta, int32_t n, double alpha, double kappa, double tol,
                              int32_t precision, double* phi, double* rms, int32_t* cycles,
                              hipStream_t stream) {
    vmg_grid g;
    std::memset(&g, 0, sizeof(g));
    g.n[0] = g.n[1] = g.n[2] = n;
    g.bc = VMG_PERIODIC;
    g.h = n > 0 ? 1.0 / n : 0.0;
    vmg_params p;
    std::memset(&p, 0, sizeof(p));
    p.alpha = alpha;
    p.kappa = kappa;
    p.tol = tol;
    p.max_cycles = 200;
    p.prec = precision;
    vmg_plan* plan = nullptr;
    vmg_status st = vmg_plan_create(&plan, &g, 1, &p, stream);
    if (st != VMG_OK) return st;
    vmg_result r;
    std::memset(&r, 0, sizeof(r));
    st = vmg_solve(plan, delta, nullptr, nullptr, phi, &r);
    std::string msg = g_err;
    vmg_plan_destroy(plan);
    g_err = msg;
    if (rms) *rms = r.rms;
    if (cycles) *cycles = r.cycles;
    return st;
}

// Multilevel plans: the domain grid, then every depth of the refinement tree
// as one batched plan; a solve fills each refinement's ghost shell and initial
// guess from its parent's solution before solving that depth.
struct vmg_levels {
    std::vector<vmg_grid> grids;
    std::vector<vmg_nest> nest;
    std::vector<std::vector<int>> members;     // grid indices per depth
    std::vector<vmg_plan*> plans;              // one per depth
    hipStream_t stream = nullptr;
};

static vmg_status levels_check(const vmg_grid* grids, const vmg_nest* nest, int32_t n_grids, std::vector<int>& depth) {
    if (!grids || !nest || n_grids < 1) return fail(VMG_EINVAL, "null argument");
    if (nest[0].parent != -1 || grids[0].bc != VMG_PERIODIC)
        return fail(VMG_EINVAL, "grid 0 must be the periodic domain grid (parent -1)");
    depth.assign(n_grids, 0);
    for (int i = 1; i < n_grids; ++i) {
        const int pa = nest[i].parent;
        if (pa < 0 || pa >= i)
            return fail(VMG_EINVAL, "grid " + std::to_string(i) + ": the parent must be an earlier grid");
        const vmg_grid& g = grids[i];
        const vmg_grid& P = grids[pa];
        if (g.bc != VMG_DIRICHLET) return fail(VMG_EINVAL, "grid " + std::to_string(i) + ": refinements are Dirichlet");
        if (!(std::fabs(2.0 * g.h - P.h) <= 1e-12 * P.h))
            return fail(VMG_EINVAL, "grid " + std::to_string(i) + ": a refinement halves its parent's cell size");
        for (int d = 0; d < 3; ++d) {
            const int o = nest[i].origin[d];
            const bool ok = P.bc == VMG_PERIODIC ? (o >= 0 && o < 2 * P.n[d])
                                                 : (o >= 2 && o + g.n[d] <= 2 * P.n[d] - 2);
            if (!ok)
                return fail(VMG_EINVAL, "grid " + std::to_string(i) +
                                            ": origin outside the parent (a refinement parent needs one cell of margin)");
        }
        depth[i] = depth[pa] + 1;
    }
    return VMG_OK;
}

vmg_status vmg_levels_create(vmg_levels** out, const vmg_grid* grids, const vmg_nest* nest, int32_t n_grids,
                             const vmg_params* p, hipStream_t stream) {
    g_err.clear();
    if (!out || !p) return fail(VMG_EINVAL, "null argument");
    *out = nullptr;
    std::vector<int> depth;
    vmg_status st = levels_check(grids, nest, n_grids, depth);
    if (st != VMG_OK) return st;
    vmg_levels* L = new (std::nothrow) vmg_levels();
    if (!L) return fail(VMG_ENOMEM, "host allocation failed");
    L->grids.assign(grids, grids + n_grids);
    L->nest.assign(nest, nest + n_grids);
    L->stream = stream;
    const int max_depth = *std::max_element(depth.begin(), depth.end());
    L->members.resize(max_depth + 1);
    for (int i = 0; i < n_grids; ++i) L->members[depth[i]].push_back(i);
    vmg_params pr = *p;
    for (int d = 0; d <= max_depth; ++d) {
        std::vector<vmg_grid> sub;
        for (int i : L->members[d]) sub.push_back(grids[i]);
        vmg_plan* plan = nullptr;
        st = vmg_plan_create(&plan, sub.data(), (int32_t)sub.size(), &pr, stream);
        if (st != VMG_OK) {
            const std::string msg = g_err;
            vmg_levels_destroy(L);
            g_err = msg;
            return st;
        }
        L->plans.push_back(plan);
    }
    *out = L;
    return VMG_OK;
}

vmg_status vmg_levels_solve(vmg_levels* L, const double* delta, double* ghost, double* phi, vmg_result* out) {
    g_err.clear();
    if (!L || !delta || !phi || !out) return fail(VMG_EINVAL, "null argument");
    if (L->grids.size() > 1 && !ghost) return fail(VMG_EINVAL, "refinements need a ghost array");
    for (size_t i = 0; i < L->grids.size(); ++i) std::memset(&out[i], 0, sizeof(vmg_result));   // unsolved levels stay 0
    for (size_t d = 0; d < L->plans.size(); ++d) {
        const std::vector<int>& idx = L->members[d];
        if (d > 0)
            for (int i : idx) {
                const vmg_grid& g = L->grids[i];
                const vmg_grid& P = L->grids[L->nest[i].parent];
                const int* o = L->nest[i].origin;
                CKH(launch_ghost_fill(phi + P.offset, P.n[0], P.n[1], P.n[2], P.h, g.n[0], g.n[1], g.n[2], g.h, o[0],
                                      o[1], o[2], ghost + g.ghost_offset, L->stream));
                CKH(launch_interior_fill(phi + P.offset, P.n[0], P.n[1], P.n[2], P.h, g.n[0], g.n[1], g.n[2], g.h,
                                         o[0], o[1], o[2], phi + g.offset, L->stream));
            }
        std::vector<vmg_result> res(idx.size());
        const vmg_status st = vmg_solve(L->plans[d], delta, d > 0 ? ghost : nullptr, nullptr, phi, res.data());
        for (size_t k = 0; k < idx.size(); ++k) out[idx[k]] = res[k];
        if (st != VMG_OK) return st;
    }
    return VMG_OK;
}

void vmg_levels_destroy(vmg_levels* L) {
    if (!L) return;
    for (vmg_plan* p : L->plans) vmg_plan_destroy(p);
    delete L;
}

vmg_status vmg_solve_levels(const vmg_grid* grids, const vmg_nest* nest, int32_t n_grids, const vmg_params* p,
                            const double* delta, double* ghost, double* phi, vmg_result* out, hipStream_t stream) {
    g_err.clear();
    if (!delta || !phi || !out) return fail(VMG_EINVAL, "null argument");
    if (n_grids > 1 && !ghost) return fail(VMG_EINVAL, "refinements need a ghost array");
    vmg_levels* L = nullptr;
    vmg_status st = vmg_levels_create(&L, grids, nest, n_grids, p, stream);
    if (st != VMG_OK) return st;
    st = vmg_levels_solve(L, delta, ghost, phi, out);
    const std::string msg = g_err;
    vmg_levels_destroy(L);
    g_err = msg;
    return st;
}

vmg_status vmg_residual(vmg_plan* plan, int32_t gi, const double* delta, const double* ghost,
                        const double* source, const double* phi, double* d, vmg_result* res) {
    g_err.clear();
    if (!plan || !delta || !phi) return fail(VMG_EINVAL, "null plan, delta or phi");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (gi < 0 || gi >= (int)P->grids.size()) return fail(VMG_EINVAL, "grid index out of range");
    GridState& G = P->grids[gi];
    LevelBuf& L0 = G.lev[0];
    if (L0.g.dir && !ghost) return fail(VMG_EINVAL, "Dirichlet grids need ghost values");
    hipStream_t s = P->stream;
    const bool had = P->has_source;
    P->has_source = source != nullptr;
    L0.cur = 0;
    CKH(launch_copy_in(L0.g, delta + G.desc.offset, L0.delta, s));
    CKH(launch_copy_in(L0.g, phi + G.desc.offset, L0.phi[0], s));
    if (source) CKH(launch_copy_in(L0.g, source + G.desc.offset, L0.f, s));
    if (L0.g.dir) CKH(launch_ghost_in(L0.g, ghost + G.desc.ghost_offset, L0.phi[0], s));
    CKH(launch_fill((double*)L0.sc, sizeof(LevelScalars) / sizeof(double), 0.0, s));
    int nb = 0;
    const double* f = P->has_source ? L0.f : nullptr;
    // first pass sets cbar, second evaluates d with it
    CKH(launch_residual_norm(L0.g, P->coef, L0.phi[0], L0.delta, f, L0.sc, nullptr, P->partials, &nb, s));
    CKH(launch_finalize(P->partials, nb, L0.g.ncell, L0.g.dir ? 0 : 1, 0, L0.sc, G.norm_dev, s));
    CKH(launch_residual_norm(L0.g, P->coef, L0.phi[0], L0.delta, f, L0.sc, d ? d + G.desc.offset : nullptr,
                             P->partials, &nb, s));
    CKH(launch_finalize(P->partials, nb, L0.g.ncell, L0.g.dir ? 0 : 1, 0, L0.sc, G.norm_dev, s));
    NormOut no;
    CKH(hipMemcpyAsync(&no, G.norm_dev, sizeof(NormOut), hipMemcpyDeviceToHost, s));
    CKH(hipStreamSynchronize(s));
    P->has_source = had;
    P->solved = false;   // the finest-level buffers no longer hold a solve's state
    if (res) {
        res->rms0 = no.rms;
        res->rms = no.rms;
        res->compat_c = no.cbar;
        res->cycles = 0;
        res->inner_cycles = 0;
        res->n_guarded = (int64_t)no.n_guard;
    }
    return VMG_OK;
}

vmg_status vmg_fill_ghosts(const double* parent, const int32_t np[3], double parent_h, const vmg_grid* grids,
                           const int32_t* origins, int32_t n_grids, double* ghost, hipStream_t stream) {
    g_err.clear();
    if (!parent || !np || !grids || !origins || !ghost || n_grids < 1)
        return fail(VMG_EINVAL, "null argument");
    if (np[0] < 1 || np[1] < 1 || np[2] < 1 || !(parent_h > 0.0)) return fail(VMG_EINVAL, "bad parent grid");
    for (int i = 0; i < n_grids; ++i) {
        const vmg_grid& g = grids[i];
        if (g.bc != VMG_DIRICHLET || g.n[0] < 1 || g.n[1] < 1 || g.n[2] < 1 || !(g.h > 0.0))
            return fail(VMG_EINVAL, "ghost fill needs Dirichlet grids with n >= 1 and h > 0");
        CKH(launch_ghost_fill(parent, np[0], np[1], np[2], parent_h, g.n[0], g.n[1], g.n[2], g.h,
                              origins[3 * i], origins[3 * i + 1], origins[3 * i + 2], ghost + g.ghost_offset,
                              stream));
    }
    return VMG_OK;
}

vmg_status vmg_fill_interior(const double* parent, const int32_t np[3], double parent_h, const vmg_grid* grids,
                             const int32_t* origins, int32_t n_grids, double* phi, hipStream_t stream) {
    g_err.clear();
    if (!parent || !np || !grids || !origins || !phi || n_grids < 1) return fail(VMG_EINVAL, "null argument");
    if (np[0] < 1 || np[1] < 1 || np[2] < 1 || !(parent_h > 0.0)) return fail(VMG_EINVAL, "bad parent grid");
    for (int i = 0; i < n_grids; ++i) {
        const vmg_grid& g = grids[i];
        if (g.n[0] < 1 || g.n[1] < 1 || g.n[2] < 1 || !(g.h > 0.0) || g.offset < 0)
            return fail(VMG_EINVAL, "interior fill needs grids with n >= 1, h > 0 and offset >= 0");
        CKH(launch_interior_fill(parent, np[0], np[1], np[2], parent_h, g.n[0], g.n[1], g.n[2], g.h,
                                 origins[3 * i], origins[3 * i + 1], origins[3 * i + 2], phi + g.offset, stream));
    }
    return VMG_OK;
}

vmg_status vmg_total_force(const double* phi_newton, const double* phi, const int32_t n[3], double h, double* psi,
                           double* force, hipStream_t stream) {
    g_err.clear();
    if (!phi_newton || !phi || !n || !force) return fail(VMG_EINVAL, "null argument");
    if (n[0] < 1 || n[1] < 1 || n[2] < 1 || !(h > 0.0) || !std::isfinite(h) ||
        total_force_blocks(n[0], n[1], n[2]) > INT32_MAX)
        return fail(VMG_EINVAL, "total force needs n >= 1 per axis, a grid of fewer than 2^31 tiles and a finite h > 0");
    CKH(launch_total_force(n[0], n[1], n[2], h, phi_newton, phi, psi, force, stream));
    return VMG_OK;
}

static bool assign_args_ok(int64_t n_particles, const int32_t n[3]) {
    return n && n_particles >= 1 && n_particles <= INT32_MAX && n[0] >= 1 && n[1] >= 1 && n[2] >= 1 &&
           n[1] <= 65535 && n[2] <= 65535 &&
           mass_assign_bricks(n[0], n[1], n[2]) <= (int64_t(1) << 26);
}

int64_t vmg_mass_assign_workspace(int64_t n_particles, const int32_t n[3]) {
    if (!assign_args_ok(n_particles, n)) return -1;
    return mass_assign_workspace(n_particles, n[0], n[1], n[2]);
}

vmg_status vmg_mass_assign(const double* pos, int64_t n_particles, const int32_t n[3], int32_t scheme,
                           void* workspace, int64_t workspace_bytes, double* delta, hipStream_t stream) {
    g_err.clear();
    if (!pos || !n || !delta || !workspace) return fail(VMG_EINVAL, "null argument");
    if (n_particles < 1 || n_particles > INT32_MAX)
        return fail(VMG_EINVAL, "mass assignment needs 1 <= n_particles <= 2^31 - 1");
    if (!assign_args_ok(n_particles, n)) return fail(VMG_EINVAL, "mass assignment needs n >= 1 per axis");
    if (scheme != VMG_ASSIGN_CIC && scheme != VMG_ASSIGN_TSC) return fail(VMG_EINVAL, "unknown assignment scheme");
    if (workspace_bytes < mass_assign_workspace(n_particles, n[0], n[1], n[2]) ||
        reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(VMG_EINVAL, "mass assignment workspace too small or not 256-byte aligned");
    const double mean_count = (double)n_particles / ((double)n[0] * n[1] * n[2]);
    CKH(launch_mass_assign(pos, n_particles, n[0], n[1], n[2], scheme, true, 0.0, nullptr, mean_count, workspace,
                           delta, stream));
    return VMG_OK;
}

vmg_status vmg_mass_assign_noalloc(const double* pos, int64_t n_particles, const int32_t n[3], int32_t scheme,
                                   double* delta, hipStream_t stream) {
    g_err.clear();
    if (!pos || !n || !delta) return fail(VMG_EINVAL, "null argument");
    if (n_particles < 1 || n_particles > INT32_MAX)
        return fail(VMG_EINVAL, "mass assignment needs 1 <= n_particles <= 2^31 - 1");
    if (!assign_args_ok(n_particles, n)) return fail(VMG_EINVAL, "mass assignment needs n >= 1 per axis");
    if (scheme != VMG_ASSIGN_CIC && scheme != VMG_ASSIGN_TSC) return fail(VMG_EINVAL, "unknown assignment scheme");
    const int64_t need = mass_assign_workspace(n_particles, n[0], n[1], n[2]);
    if (need > NOALLOC_SCRATCH_BYTES)
        return fail(VMG_EINVAL, "vmg_mass_assign_noalloc: the workspace this call needs (" + std::to_string(need) +
                                    " bytes) exceeds the static scratch of " +
                                    std::to_string(NOALLOC_SCRATCH_BYTES) + " bytes");
    void* work = nullptr;
    CKH(noalloc_scratch(&work));
    const double mean_count = (double)n_particles / ((double)n[0] * n[1] * n[2]);
    CKH(launch_mass_assign(pos, n_particles, n[0], n[1], n[2], scheme, true, 0.0, nullptr, mean_count, work, delta,
                           stream));
    return VMG_OK;
}

vmg_status vmg_mass_assign_region(const double* pos, int64_t n_particles, const int32_t n[3], double h,
                                  const double corner[3], double mean_count, int32_t scheme, void* workspace,
                                  int64_t workspace_bytes, double* delta, hipStream_t stream) {
    g_err.clear();
    if (!pos || !n || !corner || !delta || !workspace) return fail(VMG_EINVAL, "null argument");
    if (n_particles < 1 || n_particles > INT32_MAX)
        return fail(VMG_EINVAL, "mass assignment needs 1 <= n_particles <= 2^31 - 1");
    if (!assign_args_ok(n_particles, n)) return fail(VMG_EINVAL, "mass assignment needs n >= 1 per axis");
    if (!(h > 0.0) || !std::isfinite(h) || !(mean_count > 0.0) || !std::isfinite(mean_count))
        return fail(VMG_EINVAL, "region assignment needs a finite h > 0 and mean_count > 0");
    for (int a = 0; a < 3; ++a) {
        if (!std::isfinite(corner[a])) return fail(VMG_EINVAL, "region corner must be finite");
        if (!(n[a] * h <= 1.0 - 4.0 * h))
            return fail(VMG_EINVAL, "a region must leave at least 4 of its cells of the box uncovered per axis");
    }
    if (scheme != VMG_ASSIGN_CIC && scheme != VMG_ASSIGN_TSC) return fail(VMG_EINVAL, "unknown assignment scheme");
    if (workspace_bytes < mass_assign_workspace(n_particles, n[0], n[1], n[2]) ||
        reinterpret_cast<uintptr_t>(workspace) % 256 != 0)
        return fail(VMG_EINVAL, "mass assignment workspace too small or not 256-byte aligned");
    CKH(launch_mass_assign(pos, n_particles, n[0], n[1], n[2], scheme, false, h, corner, mean_count, workspace, delta,
                           stream));
    return VMG_OK;
}

vmg_status vmg_smooth(vmg_plan* plan, int32_t sweeps) {
    g_err.clear();
    if (!plan || sweeps < 0) return fail(VMG_EINVAL, "null plan or sweeps < 0");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (!P->solved) return fail(VMG_EINVAL, "vmg_smooth needs a previous vmg_solve");
    for (int s = 0; s < sweeps; ++s) {
        if (P->batched) {
            CKH(batch_smooth_finest(P));
            continue;
        }
        for (auto& G : P->grids) CKH(P->mixed ? smooth_corr_level(P, G, 0) : smooth_level(P, G, 0));
    }
    return VMG_OK;
}

vmg_status vmg_plan_set_schedule(vmg_plan* plan, int32_t level, int32_t tile_y, int32_t z_chunk, int32_t pipe) {
    g_err.clear();
    if (!plan) return fail(VMG_EINVAL, "null plan");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (tile_y != 4 && tile_y != 8 && tile_y != 12 && tile_y != 16)
        return fail(VMG_EINVAL, "tile_y must be 4, 8, 12 or 16");
    if (z_chunk < 2 || z_chunk > 1024 || (z_chunk & 1)) return fail(VMG_EINVAL, "z_chunk must be even, in [2, 1024]");
    if (pipe != 0 && pipe != 1 && pipe != PIPE_BRICK) return fail(VMG_EINVAL, "pipe must be 0, 1 or 2");
    if (level < 0 || level >= swept_level_count(P))
        return fail(VMG_EINVAL, "level " + std::to_string(level) + " has no fused sweep in this plan");
    if (pipe == PIPE_BRICK && level == 0 && !P->batched)
        return fail(VMG_EINVAL, "pipe 2 (bricks) runs on the coarser levels of a periodic plan or on any level of "
                                "a Dirichlet batch");
    const SmoothCfg c{tile_y, z_chunk, pipe};
    if (level == 0) P->cfg = c;
    if (P->batched) {
        CKH(batch_set_level_cfg(P, level, c));
    } else if (level > 0) {
        if ((int)P->lcfg.size() < (int)P->grids[0].lev.size())
            P->lcfg.resize(P->grids[0].lev.size(), SmoothCfg{0, 0, 1});
        P->lcfg[level] = c;
    }
    CKH(hipStreamSynchronize(P->stream));
    return capture_graphs(P);
}

vmg_status vmg_plan_schedule(const vmg_plan* plan, int32_t level, int32_t* tile_y, int32_t* z_chunk, int32_t* pipe) {
    if (!plan) return fail(VMG_EINVAL, "null plan");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (level < 0 || level >= swept_level_count(P))
        return fail(VMG_EINVAL, "level " + std::to_string(level) + " has no fused sweep in this plan");
    const SmoothCfg c = P->batched ? P->blev[level].cfg : level_schedule(P, level, P->grids[0].lev[level].g);
    if (tile_y) *tile_y = c.ty;
    if (z_chunk) *z_chunk = c.zc;
    if (pipe) *pipe = c.pipe;
    return VMG_OK;
}

vmg_status vmg_plan_time_sweeps(vmg_plan* plan, int32_t enable) {
    g_err.clear();
    if (!plan) return fail(VMG_EINVAL, "null plan");
    Plan* P = reinterpret_cast<Plan*>(plan);
    CKH(hipStreamSynchronize(P->stream));
    if (enable && P->tev.empty()) {
        P->tev.assign(2 * 256, nullptr);
        P->tev_count.assign(256, 0);
        for (auto& ev : P->tev) CKH(hipEventCreate(&ev));
    }
    P->time_sweeps = enable != 0;
    P->sweep_us = 0.0;
    P->sweep_n = 0;
    P->tev_used = 0;
    return capture_graphs(P);
}

vmg_status vmg_plan_sweep_time(const vmg_plan* plan, double* total_us, int64_t* launches) {
    if (!plan) return fail(VMG_EINVAL, "null plan");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (total_us) *total_us = P->sweep_us;
    if (launches) *launches = P->sweep_n;
    return VMG_OK;
}

vmg_status vmg_plan_time_levels(vmg_plan* plan, int32_t enable) {
    g_err.clear();
    if (!plan) return fail(VMG_EINVAL, "null plan");
    Plan* P = reinterpret_cast<Plan*>(plan);
    CKH(hipStreamSynchronize(P->stream));
    if (enable && P->lev_ev.empty()) {
        P->lev_ev.assign(2 * 512, nullptr);
        P->lev_tag.assign(512, 0);
        for (auto& ev : P->lev_ev) CKH(hipEventCreate(&ev));
    }
    size_t nlev = 0;
    for (const auto& G : P->grids) nlev = std::max(nlev, G.lev.size());
    P->time_levels = enable != 0 && !P->batched;
    P->level_us.assign(nlev, 0.0);
    P->level_cycles = 0;
    P->lev_used = 0;
    return capture_graphs(P);
}

vmg_status vmg_plan_level_time(const vmg_plan* plan, int32_t level, double* total_us, int64_t* iterations) {
    if (!plan) return fail(VMG_EINVAL, "null plan");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    size_t nlev = 0;
    for (const auto& G : P->grids) nlev = std::max(nlev, G.lev.size());
    if (level < 0 || (size_t)level >= nlev) return fail(VMG_EINVAL, "level out of range");
    if (total_us) *total_us = (size_t)level < P->level_us.size() ? P->level_us[level] : 0.0;
    if (iterations) *iterations = P->level_cycles;
    return VMG_OK;
}

vmg_status vmg_plan_history(const vmg_plan* plan, int32_t grid, vmg_history* out, int32_t cap, int32_t* n) {
    if (!plan || !n) return fail(VMG_EINVAL, "null argument");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (grid < 0 || grid >= (int32_t)P->grids.size()) return fail(VMG_EINVAL, "grid out of range");
    if (cap < 0 || (cap > 0 && !out)) return fail(VMG_EINVAL, "bad output buffer");
    const std::vector<vmg_history> none;
    const auto& h = (size_t)grid < P->history.size() ? P->history[grid] : none;
    *n = (int32_t)h.size();
    for (int32_t i = 0; i < cap && i < (int32_t)h.size(); ++i) out[i] = h[i];
    return VMG_OK;
}

vmg_status vmg_plan_get_cycle(const vmg_plan* plan, vmg_cycle* cycle) {
    if (!plan || !cycle) return fail(VMG_EINVAL, "null argument");
    get_cycle(reinterpret_cast<const Plan*>(plan), cycle);
    return VMG_OK;
}

vmg_status vmg_plan_set_cycle(vmg_plan* plan, const vmg_cycle* cycle) {
    g_err.clear();
    if (!plan || !cycle) return fail(VMG_EINVAL, "null argument");
    return set_cycle(reinterpret_cast<Plan*>(plan), cycle);
}

vmg_status vmg_plan_tune_cycle(vmg_plan* plan, const double* delta, const double* ghost, const double* source,
                               double* phi_work, vmg_cycle* best, double* best_ms) {
    g_err.clear();
    if (!plan || !delta || !phi_work) return fail(VMG_EINVAL, "null plan, delta or phi_work");
    Plan* P = reinterpret_cast<Plan*>(plan);
    if (!P->periodic && !ghost) return fail(VMG_EINVAL, "Dirichlet grids need ghost values");
    return tune_cycle(P, delta, ghost, source, phi_work, best, best_ms);
}

int32_t vmg_plan_level_count(const vmg_plan* plan) {
    if (!plan) return -1;
    return swept_level_count(reinterpret_cast<const Plan*>(plan));
}

vmg_status vmg_plan_config(const vmg_plan* plan, int32_t* tile_y, int32_t* z_chunk, int32_t* nu1, int32_t* nu2,
                           int32_t* coarse_sweeps) {
    if (!plan) return fail(VMG_EINVAL, "null plan");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (tile_y) *tile_y = P->cfg.ty;
    if (z_chunk) *z_chunk = P->cfg.zc;
    if (nu1) *nu1 = P->nu1;
    if (nu2) *nu2 = P->nu2;
    if (coarse_sweeps) *coarse_sweeps = P->ncoarse;
    return VMG_OK;
}

vmg_status vmg_plan_stats(const vmg_plan* plan, int64_t* cell_updates, int64_t* finest_sweeps,
                          int64_t* finest_cells) {
    if (!plan) return fail(VMG_EINVAL, "null plan");
    const Plan* P = reinterpret_cast<const Plan*>(plan);
    if (cell_updates) *cell_updates = P->cell_updates;
    if (finest_sweeps) *finest_sweeps = P->finest_sweeps;
    if (finest_cells) {
        int64_t c = 0;
        for (const auto& G : P->grids) c += G.lev[0].g.ncell;
        *finest_cells = c;
    }
    return VMG_OK;
}

}  // extern "C"
