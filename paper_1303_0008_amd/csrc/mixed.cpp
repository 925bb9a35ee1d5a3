// Host side of the mixed-precision path: FP32 correction V-cycle inside an
// FP64 defect-correction loop (residual, root near a vanishing discriminant
// and norms stay FP64; smoothing, restriction and prolongation are FP32).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "vmg_internal.h"
#include "vmg_plan.h"

namespace vmg {

CoefF make_coef_f(const Coef& c, double h) {
    CoefF f;
    f.alpha = (float)c.alpha;
    f.c8 = (float)c.c8;
    f.a34 = c.alpha != 0.0 ? (float)(3.0 / (4.0 * c.alpha)) : 0.0f;
    f.a_ih4 = (float)(c.alpha / (h * h * h * h));
    f.h2 = (float)(h * h);
    return f;
}

vmg_status alloc_mixed(Plan* P) {
    hipStream_t s = P->stream;
    for (auto& G : P->grids) {
        for (size_t l = 0; l < G.lev.size(); ++l) {
            LevelBuf& L = G.lev[l];
            const size_t n = (size_t)L.g.nstore;
            float** bufs[] = {&L.e[0], &L.e[1], &L.r, &L.pt, &L.t0, &L.eold, &L.rdf};
            const int nb = l > 0 ? 7 : 5;
            for (int b = 0; b < nb; ++b) {
                if (hipMalloc((void**)bufs[b], sizeof(float) * n) != hipSuccess)
                    return fail(VMG_ENOMEM, "hipMalloc failed (mixed buffers)");
                P->allocs.push_back(*bufs[b]);
                if (launch_fill_f(*bufs[b], (int64_t)n, 0.0f, s) != hipSuccess)
                    return fail(VMG_EHIP, "fill failed");
            }
            if (hipMalloc((void**)&L.scf, sizeof(LevelScalars)) != hipSuccess)
                return fail(VMG_ENOMEM, "hipMalloc failed (mixed scalars)");
            P->allocs.push_back(L.scf);
            if (launch_fill((double*)L.scf, sizeof(LevelScalars) / sizeof(double), 0.0, s) != hipSuccess)
                return fail(VMG_EHIP, "fill failed");
        }
    }
    return VMG_OK;
}

// FP32 ghost shells of the base state (Dirichlet): cast the FP64 level arrays
// once per solve; interiors are rewritten every outer iteration.
hipError_t mixed_prepare(Plan* P) {
    hipError_t e;
    for (auto& G : P->grids)
        for (auto& L : G.lev)
            if (L.g.dir && (e = launch_cast_all(L.phi[0], L.pt, L.g.nstore, P->stream)) != hipSuccess) return e;
    return hipSuccess;
}

// `count` correction sweeps of level l (one launch per sweep, or per two on the
// brick schedule); zero_in and pro apply to the first
hipError_t smooth_corr_level_n(Plan* P, GridState& G, int l, int count, bool zero_in, const ProlongInF* pro) {
    LevelBuf& L = G.lev[l];
    const CoefF cf = make_coef_f(P->coef, L.g.h);
    const SmoothCfg cfg = level_schedule(P, l, L.g);
    const int per = cfg.pipe == PIPE_BRICK ? 2 : 1;
    for (int s = 0; s < count;) {
        const int n = std::min(per, count - s);
        hipError_t e = launch_smooth_corr(L.g, cf, L.e[L.ecur], L.e[L.ecur ^ 1], L.pt, L.t0, L.r, L.scf, cfg,
                                          P->stream, zero_in && s == 0, s == 0 ? pro : nullptr, n);
        L.ecur ^= 1;
        P->cell_updates += n * L.g.ncell;
        if (l == 0) P->finest_sweeps += n;
        if (e != hipSuccess) return e;
        s += n;
    }
    return hipSuccess;
}

hipError_t smooth_corr_level(Plan* P, GridState& G, int l, bool zero_in, const ProlongInF* pro) {
    return smooth_corr_level_n(P, G, l, 1, zero_in, pro);
}

// e^h += P(e^H - e^H_old), then nu2 correction sweeps of level l: on periodic
// grids the prolongation is folded into the first sweep where that pays (on the
// finest level that sweep is not timed with the plain ones)
hipError_t post_smooth_corr(Plan* P, GridState& G, int l, int nu2) {
    LevelBuf& L = G.lev[l];
    LevelBuf& C = G.lev[l + 1];
    hipError_t e;
    const int s0 = nu2 > 0 && fold_prolong_here(P, L.g, C.g, level_schedule(P, l, L.g)) ? 1 : 0;
    const ProlongInF pro{C.g, C.e[C.ecur], C.eold};
    if (!s0 && (e = launch_prolong_corr(L.g, C.g, L.e[L.ecur], C.e[C.ecur], C.eold, P->stream)) != hipSuccess)
        return e;
    if (l > 0) return smooth_corr_level_n(P, G, l, nu2, false, s0 ? &pro : nullptr);
    if (s0 && (e = smooth_corr_level(P, G, l, false, &pro)) != hipSuccess) return e;
    if ((e = sweep_mark(P, true, nu2 - s0)) != hipSuccess) return e;
    if ((e = smooth_corr_level_n(P, G, l, nu2 - s0, false, nullptr)) != hipSuccess) return e;
    return sweep_mark(P, false, nu2 - s0);
}

// The periodic coarse tail of the inner cycle: levels l..last in one launch.
static hipError_t inner_tail(Plan* P, GridState& G, int l) {
    const int last = (int)G.lev.size() - 1;
    TailCorrArgs a;
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
    a.e = L.e[L.ecur];
    a.r = L.r;
    a.pt = L.pt;
    a.t0 = L.t0;
    a.sc = L.scf;
    a.c64 = P->coef;
    a.nu1 = pre_sweeps(P, l); a.nu2 = post_sweeps(P, l); a.ncoarse = P->ncoarse;
    return launch_tail_corr(a, P->stream);
}

// zero_e: the level's correction is identically zero on entry (finest level,
// first inner cycle of an outer iteration); the first sweep then reads no e.
// fresh_base: the first inner cycle of an outer iteration restricts the base
// state phi~ and computes the coarse t0; later inner cycles of the same outer
// iteration reuse them (phi~ only changes in the outer FP64 pass).
static hipError_t inner_vcycle(Plan* P, GridState& G, int l, bool zero_e, bool fresh_base) {
    LevelBuf& L = G.lev[l];
    const int last = (int)G.lev.size() - 1;
    const CoefF cf = make_coef_f(P->coef, L.g.h);
    hipError_t e;
    if (l > 0 && l == tail_level(P, G)) {
        if ((e = level_mark(P, l, true)) != hipSuccess || (e = inner_tail(P, G, l)) != hipSuccess) return e;
        return level_mark(P, l, false);
    }
    if (l == last) {
        if ((e = level_mark(P, l, true)) != hipSuccess) return e;
        e = launch_coarse_corr(L.g, cf, L.e[L.ecur], L.pt, L.t0, L.r, P->ncoarse, P->stream);
        P->cell_updates += (int64_t)P->ncoarse * L.g.ncell;
        if (e != hipSuccess) return e;
        return level_mark(P, l, false);
    }
    if ((e = level_mark(P, l, true)) != hipSuccess) return e;
    // the sweep that reads no correction (zero_e) is another kernel: it is not timed
    const int nu1 = pre_sweeps(P, l);
    const int t1 = zero_e ? nu1 - 1 : nu1;
    if (l > 0) {
        if ((e = smooth_corr_level_n(P, G, l, nu1, zero_e)) != hipSuccess) return e;
    } else {
        for (int s = 0; s < nu1; ++s) {
            if (s == nu1 - t1 && (e = sweep_mark(P, true, t1)) != hipSuccess) return e;
            if ((e = smooth_corr_level(P, G, l, zero_e && s == 0)) != hipSuccess) return e;
        }
        if (t1 > 0 && (e = sweep_mark(P, false, t1)) != hipSuccess) return e;
    }
    LevelBuf& C = G.lev[l + 1];
    const CoefF cc = make_coef_f(P->coef, C.g.h);
    C.ecur = 0;
    int nb = 0;
    const int periodic = L.g.dir ? 0 : 1;
    // restriction of e and d_e; the coarse base state phi~ is restricted in the same pass
    if ((e = launch_rr_corr(L.g, C.g, cf, L.e[L.ecur], L.pt, L.t0, L.r, L.scf, C.e[0], C.eold, C.rdf,
                            fresh_base ? C.pt : nullptr, P->partials, &nb, P->stream)) != hipSuccess)
        return e;
    // coarse rhs; also the coarse t0 (FP64 discriminant of the restricted base state)
    int nbc = 0;
    if ((e = launch_fas_corr(C.g, cc, P->coef, C.delta, C.e[0], C.pt, C.t0, C.rdf, C.r, P->partials_b, &nbc,
                             P->stream, fresh_base)) != hipSuccess)
        return e;
    // cbar of level l's correction equation (its post-smoothing) and of level l+1
    if (periodic &&
        (e = launch_finalize_pair(FinJob{P->partials, nb, 1, 0, L.g.ncell, L.scf, nullptr, nullptr},
                                  FinJob{P->partials_b, nbc, 1, 1, C.g.ncell, C.scf, nullptr, nullptr},
                                  P->stream)) != hipSuccess)
        return e;
    if ((e = level_mark(P, l, false)) != hipSuccess) return e;
    if ((e = inner_vcycle(P, G, l + 1, false, fresh_base)) != hipSuccess) return e;
    if ((e = level_mark(P, l, true)) != hipSuccess) return e;
    if ((e = post_smooth_corr(P, G, l, post_sweeps(P, l))) != hipSuccess) return e;
    return level_mark(P, l, false);
}

static const double* level0_f(const Plan* P, const GridState& G) {
    return P->has_source ? G.lev[0].f : nullptr;
}

// FP64 residual of phi (after adding the correction e when `update`), FP32
// inputs of the inner problem and the norm.  With `update` phi ping-pongs.
static hipError_t cast_pass(Plan* P, GridState& G, bool update) {
    LevelBuf& L = G.lev[0];
    int nb = 0;
    hipError_t e = level_mark(P, 0, true);
    if (e != hipSuccess) return e;
    e = launch_cast_update(L.g, P->coef, L.phi[L.cur], update ? L.e[L.ecur] : nullptr, L.phi[L.cur ^ 1],
                           L.delta, level0_f(P, G), L.sc, L.pt, L.t0, L.r, P->partials, &nb, P->stream);
    if (e != hipSuccess) return e;
    if (update) L.cur ^= 1;
    if ((e = launch_finalize(P->partials, nb, L.g.ncell, L.g.dir ? 0 : 1, 2, L.sc, G.norm_dev, P->stream,
                             L.scf)) != hipSuccess)
        return e;
    return level_mark(P, 0, false);
}

// Truncation-error estimate tau^h = L^H(R phi) - R L^h(phi) of the current FP64
// phi (Sec. III.C) into the grid's NormOut, for plans that stop on it: the FP64
// head passes of a cycle (restriction of phi and d, coarse right-hand side with
// its tau sums) over level 1, whose FP64 buffers the mixed path leaves unused.
static hipError_t tau_pass(Plan* P, GridState& G) {
    LevelBuf& L = G.lev[0];
    LevelBuf& C = G.lev[1];
    int nb = 0, nbc = 0;
    hipError_t e = launch_residual_restrict(L.g, C.g, P->coef, L.phi[L.cur], L.delta, level0_f(P, G), L.sc,
                                            C.phi[0], C.phiold, C.rd, P->partials, &nb, P->stream);
    if (e != hipSuccess) return e;
    if ((e = launch_fas_rhs(C.g, P->coef, C.phi[0], C.delta, C.rd, C.f, P->partials_b, &nbc, P->stream,
                            level0_f(P, G), &L.g)) != hipSuccess)
        return e;
    return launch_finalize(P->partials_b, nbc, C.g.ncell, C.g.dir ? 0 : 1, 1, C.sc, G.norm_dev, P->stream);
}

static hipError_t norms_to_host(Plan* P) {
    for (size_t gi = 0; gi < P->grids.size(); ++gi) {
        hipError_t e = hipMemcpyAsync(&P->host_norm[gi], P->grids[gi].norm_dev, sizeof(NormOut),
                                      hipMemcpyDeviceToHost, P->stream);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

hipError_t mixed_initial_pass(Plan* P) {
    hipError_t e;
    for (auto& G : P->grids)
        if ((e = cast_pass(P, G, false)) != hipSuccess) return e;
    return norms_to_host(P);
}

hipError_t enqueue_outer(Plan* P) {
    hipError_t e;
    for (auto& G : P->grids) {
        // the coarse base states (phi~, t0) of the inner problem are produced by the
        // restriction and coarse-rhs passes of the inner cycle's descent
        LevelBuf& L0 = G.lev[0];
        L0.ecur = 0;
        const bool zero_e = P->nu1 > 0 && G.lev.size() > 1;
        if (!zero_e && (e = launch_fill_f(L0.e[0], L0.g.nstore, 0.0f, P->stream)) != hipSuccess) return e;
        for (int c = 0; c < P->inner; ++c)
            if ((e = inner_vcycle(P, G, 0, zero_e && c == 0, c == 0)) != hipSuccess) return e;
        if ((e = cast_pass(P, G, true)) != hipSuccess) return e;
        if (P->params.tau_factor > 0.0 && (e = tau_pass(P, G)) != hipSuccess) return e;
    }
    return norms_to_host(P);
}

}  // namespace vmg
