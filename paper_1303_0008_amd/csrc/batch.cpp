// Batched Dirichlet grids (refinement patches, Sec. III.C and IV.D): every grid
// of a plan shares pooled per-level buffers, and each multigrid step is one
// launch per level over a work list that spans all grids (persistent smoother
// over (grid, tile, z-chunk) items; 256-cell blocks for the other passes).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstring>
#include <string>
#include <vector>

#include "vmg_internal.h"
#include "vmg_plan.h"

namespace vmg {

#define CKE(expr)                                 \
    do {                                          \
        hipError_t _e = (expr);                   \
        if (_e != hipSuccess) return _e;          \
    } while (0)

template <typename T>
static hipError_t upload(Plan* P, T** dst, const std::vector<T>& v) {
    *dst = nullptr;
    if (v.empty()) return hipSuccess;
    CKE(hipMalloc((void**)dst, sizeof(T) * v.size()));
    P->allocs.push_back(*dst);
    return hipMemcpy(*dst, v.data(), sizeof(T) * v.size(), hipMemcpyHostToDevice);
}

static void cell_items(std::vector<int2>& out, int k, int64_t n) {
    for (int64_t s = 0; s < n; s += ITEM_CELLS) out.push_back(make_int2(k, (int)s));
}

// Work list of the persistent smoother on level l for schedule cfg (the grids of
// the level that continue below it).
hipError_t batch_set_level_cfg(Plan* P, int l, SmoothCfg cfg) {
    BatchLevel& B = P->blev[l];
    B.cfg = cfg;
    std::vector<int4> items;
    for (size_t k = 0; k < B.members.size(); ++k) {
        if (B.coarsest[k]) continue;
        const Geom& g = P->grids[B.members[k]].lev[l].g;
        if (cfg.pipe == PIPE_BRICK) {   // (grid, brick x, brick y, brick z)
            const int bx = (g.n0 + BB_SIDE - 1) / BB_SIDE, by = (g.n1 + BB_SIDE - 1) / BB_SIDE;
            const int bz = (g.n2 + BB_SIDE - 1) / BB_SIDE;
            for (int z = 0; z < bz; ++z)
                for (int y = 0; y < by; ++y)
                    for (int x = 0; x < bx; ++x) items.push_back(make_int4((int)k, x, y, z));
            continue;
        }
        const int tx = (g.n0 + TX - 1) / TX, ty = (g.n1 + cfg.ty - 1) / cfg.ty;
        const int tz = (g.n2 + cfg.zc - 1) / cfg.zc;
        for (int c = 0; c < tz; ++c)
            for (int y = 0; y < ty; ++y)
                for (int x = 0; x < tx; ++x) items.push_back(make_int4((int)k, x, y, c));
    }
    B.nsitems = (int)items.size();
    return upload(P, &B.d_sitems, items);
}

// Default work lists: the finest level uses the plan's schedule; coarser levels
// shorten the z chunk, then the tile height, until the level has at least
// MIN_TILED_BLOCKS items (or the shortest schedule).
hipError_t batch_build_smooth_items(Plan* P) {
    for (size_t l = 0; l < P->blev.size(); ++l) {
        const BatchLevel& B = P->blev[l];
        auto count = [&](const SmoothCfg& c) {
            int64_t n = 0;
            for (size_t k = 0; k < B.members.size(); ++k) {
                if (B.coarsest[k]) continue;
                const Geom& g = P->grids[B.members[k]].lev[l].g;
                n += (int64_t)((g.n0 + TX - 1) / TX) * ((g.n1 + c.ty - 1) / c.ty) * ((g.n2 + c.zc - 1) / c.zc);
            }
            return n;
        };
        SmoothCfg cfg = P->cfg;
        if (l > 0) {
            while (cfg.zc > 2 && count(cfg) < MIN_TILED_BLOCKS) cfg.zc >>= 1;
            if (count(cfg) < MIN_TILED_BLOCKS && cfg.ty > 4) cfg.ty = 4;
        }
        CKE(batch_set_level_cfg(P, (int)l, cfg));
    }
    return hipSuccess;
}

// Pools, per-level geometry lists and work lists.  Called from build_plan for
// Dirichlet plans after the per-grid hierarchies (geometries only) exist.
vmg_status build_batch(Plan* P) {
    int nlev = 0;
    for (auto& G : P->grids) nlev = std::max(nlev, (int)G.lev.size());
    P->blev.assign(nlev, BatchLevel());
    const bool mixed = P->mixed;
    for (int l = 0; l < nlev; ++l) {
        BatchLevel& B = P->blev[l];
        int64_t base = 0;
        for (size_t gi = 0; gi < P->grids.size(); ++gi) {
            GridState& G = P->grids[gi];
            if ((int)G.lev.size() <= l) continue;
            Geom& g = G.lev[l].g;
            g.base = base;
            g.off0 += base;
            base += g.nstore;
            B.members.push_back((int)gi);
            B.coarsest.push_back(l == (int)G.lev.size() - 1 ? 1 : 0);
        }
        B.pool = base;
        const size_t nd = sizeof(double) * (size_t)base, nf = sizeof(float) * (size_t)base;
        double** dbuf[] = {&B.phi[0], &B.phi[1], &B.delta, &B.f, &B.phiold, &B.rd};
        for (auto pp : dbuf) {
            if (hipMalloc((void**)pp, nd) != hipSuccess) return fail(VMG_ENOMEM, "hipMalloc failed (batch pools)");
            P->allocs.push_back(*pp);
            if (launch_fill(*pp, base, 0.0, P->stream) != hipSuccess) return fail(VMG_EHIP, "fill failed");
        }
        if (mixed) {
            float** fbuf[] = {&B.e[0], &B.e[1], &B.eold, &B.r, &B.pt, &B.t0, &B.rdf};
            for (auto pp : fbuf) {
                if (hipMalloc((void**)pp, nf) != hipSuccess) return fail(VMG_ENOMEM, "hipMalloc failed (batch pools)");
                P->allocs.push_back(*pp);
                if (launch_fill_f(*pp, base, 0.0f, P->stream) != hipSuccess) return fail(VMG_EHIP, "fill failed");
            }
        }
        const int nm = (int)B.members.size();
        if (hipMalloc((void**)&B.sc, sizeof(LevelScalars) * nm) != hipSuccess ||
            (mixed && hipMalloc((void**)&B.scf, sizeof(LevelScalars) * nm) != hipSuccess))
            return fail(VMG_ENOMEM, "hipMalloc failed (batch scalars)");
        P->allocs.push_back(B.sc);
        if (mixed) P->allocs.push_back(B.scf);
        if (launch_fill((double*)B.sc, nm * (int64_t)(sizeof(LevelScalars) / sizeof(double)), 0.0, P->stream) !=
            hipSuccess)
            return fail(VMG_EHIP, "fill failed");
        if (mixed && launch_fill((double*)B.scf, nm * (int64_t)(sizeof(LevelScalars) / sizeof(double)), 0.0,
                                 P->stream) != hipSuccess)
            return fail(VMG_EHIP, "fill failed");
        // per-grid views into the pools (the single-grid kernels address a grid through its Geom)
        for (int k = 0; k < nm; ++k) {
            LevelBuf& L = P->grids[B.members[k]].lev[l];
            L.phi[0] = B.phi[0]; L.phi[1] = B.phi[1]; L.delta = B.delta; L.f = B.f;
            L.phiold = B.phiold; L.rd = B.rd;
            L.sc = B.sc + k;
            if (mixed) {
                L.e[0] = B.e[0]; L.e[1] = B.e[1]; L.eold = B.eold; L.r = B.r; L.pt = B.pt; L.t0 = B.t0;
                L.rdf = B.rdf; L.scf = B.scf + k;
            }
        }
        // geometry and work lists
        std::vector<Geom> geom, geom_fine, geomC;
        std::vector<int2> cells, store, gh;
        B.cells_A = B.cells_C = 0;
        for (int k = 0; k < nm; ++k) {
            GridState& G = P->grids[B.members[k]];
            const Geom& g = G.lev[l].g;
            geom.push_back(g);
            cell_items(cells, k, g.ncell);
            if (B.coarsest[k]) {
                geomC.push_back(g);
                B.cells_C += g.ncell;
            } else {
                B.cells_A += g.ncell;
            }
            if (l > 0) {
                const Geom& gf = G.lev[l - 1].g;
                geom_fine.push_back(gf);
                cell_items(store, k, g.nstore);
                cell_items(gh, k, ghost_count(g.n0, g.n1, g.n2));
            }
        }
        B.ncells = (int)cells.size();
        B.nstore_items = (int)store.size();
        B.nghost_items = (int)gh.size();
        B.nC = (int)geomC.size();
        if (upload(P, &B.d_geom, geom) != hipSuccess || upload(P, &B.d_geom_fine, geom_fine) != hipSuccess ||
            upload(P, &B.d_geomC, geomC) != hipSuccess || upload(P, &B.d_cells, cells) != hipSuccess ||
            upload(P, &B.d_store, store) != hipSuccess ||
            upload(P, &B.d_ghosts, gh) != hipSuccess)
            return fail(VMG_EHIP, "upload of batch work lists failed");
    }
    // level-0 extras: caller offsets, ghost items, norm block ranges
    BatchLevel& B0 = P->blev[0];
    std::vector<int64_t> uoff, goff;
    std::vector<int2> gitems;
    std::vector<int> first;
    int blk = 0;
    for (size_t k = 0; k < B0.members.size(); ++k) {
        const GridState& G = P->grids[B0.members[k]];
        uoff.push_back(G.desc.offset);
        goff.push_back(G.desc.ghost_offset);
        const Geom& g = G.lev[0].g;
        cell_items(gitems, (int)k, ghost_count(g.n0, g.n1, g.n2));
        first.push_back(blk);
        blk += (int)((g.ncell + ITEM_CELLS - 1) / ITEM_CELLS);
    }
    first.push_back(blk);
    // level-1 block ranges, for the truncation-error estimate
    std::vector<int> first1;
    if (P->blev.size() > 1 && P->blev[1].members.size() == B0.members.size()) {
        int b1 = 0;
        for (size_t k = 0; k < B0.members.size(); ++k) {
            first1.push_back(b1);
            b1 += (int)((P->grids[B0.members[k]].lev[1].g.ncell + ITEM_CELLS - 1) / ITEM_CELLS);
        }
        first1.push_back(b1);
    }
    P->bngitems = (int)gitems.size();
    if (upload(P, &P->d_uoff, uoff) != hipSuccess || upload(P, &P->d_goff, goff) != hipSuccess ||
        upload(P, &P->d_gitems, gitems) != hipSuccess || upload(P, &P->d_first, first) != hipSuccess ||
        upload(P, &P->d_first1, first1) != hipSuccess)
        return fail(VMG_EHIP, "upload of batch metadata failed");
    if (hipMalloc((void**)&P->d_norms, sizeof(NormOut) * B0.members.size()) != hipSuccess)
        return fail(VMG_ENOMEM, "hipMalloc failed (batch norms)");
    P->allocs.push_back(P->d_norms);
    if (launch_fill((double*)P->d_norms, (int64_t)B0.members.size() * (sizeof(NormOut) / sizeof(double)), 0.0,
                    P->stream) != hipSuccess)
        return fail(VMG_EHIP, "fill failed");
    if (batch_build_smooth_items(P) != hipSuccess) return fail(VMG_EHIP, "upload of smoother items failed");
    return VMG_OK;
}

int64_t batch_partials_needed(const Plan* P) {
    return P->blev.empty() ? 0 : P->blev[0].ncells + 1;
}


static const double* bf(const Plan* P, int l) {
    const BatchLevel& B = P->blev[l];
    if (l > 0) return B.f;
    return P->has_source ? B.f : nullptr;
}

// ---------------------------------------------------------------------------
// FP64 batched V-cycle
// ---------------------------------------------------------------------------
static hipError_t bsmooth(Plan* P, int l) {
    BatchLevel& B = P->blev[l];
    // below the finest level the ghosts follow the interior: the brick schedule
    // refreshes them as it writes, the march leaves that to a separate pass
    const bool fold = l > 0 && B.cfg.pipe == PIPE_BRICK;
    CKE(launch_smooth_batch_args(P->coef, B.phi[B.cur], B.phi[B.cur ^ 1], B.delta, bf(P, l), B.cfg, B.d_geom,
                                 B.d_sitems, B.nsitems, P->batch_blocks, P->stream, fold ? B.phiold : nullptr));
    B.cur ^= 1;
    P->cell_updates += B.cells_A;
    if (l == 0) P->finest_sweeps += 1;
    else if (!fold)
        CKE(launch_ghost_refresh_batch(B.d_geom, B.d_ghosts, B.nghost_items, B.phi[B.cur], B.phiold, P->stream));
    return hipSuccess;
}

static hipError_t bcycle(Plan* P, int l) {
    BatchLevel& B = P->blev[l];
    hipStream_t s = P->stream;
    if (B.nC) {
        // grids whose coarsest level is l: relax in place (result in both buffers)
        CKE(launch_coarse_batch(B.d_geomC, B.nC, P->coef, B.phi[B.cur], B.phi[B.cur ^ 1], B.delta, bf(P, l),
                                P->ncoarse, l > 0 ? B.phiold : nullptr, s));
        P->cell_updates += (int64_t)P->ncoarse * B.cells_C;
    }
    if (l + 1 >= (int)P->blev.size() || B.cells_A == 0) return hipSuccess;
    if (l == 0) CKE(sweep_mark(P, true, pre_sweeps(P, l)));
    for (int q = 0; q < pre_sweeps(P, l); ++q) CKE(bsmooth(P, l));
    if (l == 0) CKE(sweep_mark(P, false, pre_sweeps(P, l)));
    BatchLevel& C = P->blev[l + 1];
    C.cur = 0;
    CKE(launch_rr_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, P->coef, B.phi[B.cur], B.delta, bf(P, l),
                        C.phi[0], C.phiold, C.rd, s));
    CKE(launch_fas_batch(C.d_geom, C.d_cells, C.ncells, P->coef, C.phi[0], C.delta, C.rd, C.f, s));
    CKE(bcycle(P, l + 1));
    CKE(launch_prolong_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, B.phi[B.cur], C.phi[C.cur],
                             C.phiold, s));
    if (l == 0) CKE(sweep_mark(P, true, post_sweeps(P, l)));
    for (int q = 0; q < post_sweeps(P, l); ++q) CKE(bsmooth(P, l));
    if (l == 0) CKE(sweep_mark(P, false, post_sweeps(P, l)));
    return hipSuccess;
}

// Truncation-error estimate tau^h = L^H(R phi) - R L^h(phi) of every grid at the
// finest state phi (Sec. III.C) into d_norms[k].tau_rms, when the plan stops on
// it: restriction of phi and d to level 1 (as the head of a cycle), the coarse
// ghosts reset to the restricted boundary values, then the estimate.  Level 1 is
// scratch between cycles (the next head rewrites what this overwrites).
static hipError_t btau(Plan* P, const double* phi) {
    if (!(P->params.tau_factor > 0.0)) return hipSuccess;
    if (!P->d_first1) return hipErrorInvalidValue;   // plan creation requires level 1 on every grid
    BatchLevel& B = P->blev[0];
    BatchLevel& C = P->blev[1];
    hipStream_t s = P->stream;
    CKE(launch_rr_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, P->coef, phi, B.delta, bf(P, 0), C.phi[0],
                        C.phiold, C.rd, s));
    return launch_tau_batch(C.d_geom, C.d_geom_fine, C.d_cells, C.ncells, P->coef, C.phi[0], C.delta, C.rd,
                            bf(P, 0), P->partials, P->d_first1, (int)C.members.size(), P->d_norms, s);
}

static hipError_t bnorms(Plan* P) {
    BatchLevel& B = P->blev[0];
    CKE(launch_norm_batch(B.d_geom, B.d_cells, B.ncells, P->coef, B.phi[B.cur], B.delta, bf(P, 0), P->partials,
                          P->d_first, (int)B.members.size(), P->d_norms, P->stream));
    CKE(btau(P, B.phi[B.cur]));
    return hipMemcpyAsync(P->host_norm, P->d_norms, sizeof(NormOut) * B.members.size(), hipMemcpyDeviceToHost,
                          P->stream);
}

// ---------------------------------------------------------------------------
// mixed-precision batched outer iteration
// ---------------------------------------------------------------------------
static hipError_t bsmooth_corr(Plan* P, int l) {
    BatchLevel& B = P->blev[l];
    const CoefF cf = make_coef_f(P->coef, 1.0);   // per-grid h is applied inside the kernels
    const bool fold = l > 0 && B.cfg.pipe == PIPE_BRICK;   // as in bsmooth
    CKE(launch_smooth_corr_batch(cf, B.e[B.ecur], B.e[B.ecur ^ 1], B.pt, B.t0, B.r, B.cfg, B.d_geom, B.d_sitems,
                                 B.nsitems, P->batch_blocks, P->stream, fold ? B.eold : nullptr));
    B.ecur ^= 1;
    P->cell_updates += B.cells_A;
    if (l == 0) P->finest_sweeps += 1;
    else if (!fold)
        CKE(launch_ghost_refresh_batch_f(B.d_geom, B.d_ghosts, B.nghost_items, B.e[B.ecur], B.eold, P->stream));
    return hipSuccess;
}

static hipError_t bcycle_corr(Plan* P, int l) {
    BatchLevel& B = P->blev[l];
    hipStream_t s = P->stream;
    const CoefF cf = make_coef_f(P->coef, 1.0);
    if (B.nC) {
        CKE(launch_coarse_corr_batch(B.d_geomC, B.nC, cf, B.e[B.ecur], B.e[B.ecur ^ 1], B.pt, B.t0, B.r,
                                     P->ncoarse, l > 0 ? B.eold : nullptr, s));
        P->cell_updates += (int64_t)P->ncoarse * B.cells_C;
    }
    if (l + 1 >= (int)P->blev.size() || B.cells_A == 0) return hipSuccess;
    if (l == 0) CKE(sweep_mark(P, true, pre_sweeps(P, l)));
    for (int q = 0; q < pre_sweeps(P, l); ++q) CKE(bsmooth_corr(P, l));
    if (l == 0) CKE(sweep_mark(P, false, pre_sweeps(P, l)));
    BatchLevel& C = P->blev[l + 1];
    C.ecur = 0;
    CKE(launch_rr_corr_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, cf, B.e[B.ecur], B.pt, B.t0, B.r,
                             C.e[0], C.eold, C.rdf, s));
    CKE(launch_fas_corr_batch(C.d_geom, C.d_cells, C.ncells, cf, C.e[0], C.pt, C.t0, C.rdf, C.r, s));
    CKE(bcycle_corr(P, l + 1));
    CKE(launch_prolong_corr_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, B.e[B.ecur], C.e[C.ecur],
                                  C.eold, s));
    if (l == 0) CKE(sweep_mark(P, true, post_sweeps(P, l)));
    for (int q = 0; q < post_sweeps(P, l); ++q) CKE(bsmooth_corr(P, l));
    if (l == 0) CKE(sweep_mark(P, false, post_sweeps(P, l)));
    return hipSuccess;
}

static hipError_t bcast(Plan* P) {
    BatchLevel& B = P->blev[0];
    CKE(launch_cast_batch(B.d_geom, B.d_cells, B.ncells, P->coef, B.phi[0], B.delta, bf(P, 0), B.pt, B.t0, B.r,
                          P->partials, P->stream));
    CKE(launch_finalize_batch(P->partials, P->d_first, B.d_geom, (int)B.members.size(), P->d_norms, P->stream));
    CKE(btau(P, B.phi[0]));
    return hipMemcpyAsync(P->host_norm, P->d_norms, sizeof(NormOut) * B.members.size(), hipMemcpyDeviceToHost,
                          P->stream);
}

// ---------------------------------------------------------------------------
// entry points used by the driver
// ---------------------------------------------------------------------------
hipError_t batch_enqueue_iteration(Plan* P) {
    if (!P->mixed) {
        CKE(bcycle(P, 0));
        return bnorms(P);
    }
    hipStream_t s = P->stream;
    for (size_t l = 1; l < P->blev.size(); ++l) {
        BatchLevel& C = P->blev[l];
        CKE(launch_base_restrict_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, P->blev[l - 1].pt, C.pt, s));
        CKE(launch_base_t0_batch(C.d_geom, C.d_cells, C.ncells, P->coef, C.pt, C.delta, C.t0, s));
    }
    BatchLevel& B0 = P->blev[0];
    B0.ecur = 0;
    CKE(launch_fill_f(B0.e[0], B0.pool, 0.0f, s));
    for (int c = 0; c < P->inner; ++c) CKE(bcycle_corr(P, 0));
    CKE(launch_update_batch(B0.d_geom, B0.d_cells, B0.ncells, B0.phi[0], B0.e[B0.ecur], s));
    return bcast(P);
}

// Inputs -> pools, coarse densities and ghost shells, then the initial norm
// (left in host_norm after the caller synchronises).  First checks delta.
hipError_t batch_check_delta(Plan* P, const double* delta) {
    BatchLevel& B = P->blev[0];
    CKE(launch_check_finite_batch(B.d_geom, P->d_uoff, B.d_cells, B.ncells, delta, P->partials, P->stream));
    CKE(launch_finalize_batch(P->partials, P->d_first, B.d_geom, (int)B.members.size(), P->d_norms, P->stream));
    return hipMemcpyAsync(P->host_norm, P->d_norms, sizeof(NormOut) * B.members.size(), hipMemcpyDeviceToHost,
                          P->stream);
}

hipError_t batch_setup(Plan* P, const double* delta, const double* ghost, const double* source, const double* phi) {
    hipStream_t s = P->stream;
    BatchLevel& B = P->blev[0];
    B.cur = 0;
    CKE(launch_copy_in_batch(B.d_geom, P->d_uoff, B.d_cells, B.ncells, delta, B.delta, nullptr, s));
    CKE(launch_copy_in_batch(B.d_geom, P->d_uoff, B.d_cells, B.ncells, phi, B.phi[0], B.phi[1], s));
    if (source) CKE(launch_copy_in_batch(B.d_geom, P->d_uoff, B.d_cells, B.ncells, source, B.f, nullptr, s));
    CKE(launch_ghost_in_batch(B.d_geom, P->d_goff, P->d_gitems, P->bngitems, ghost, B.phi[0], B.phi[1], s));
    for (size_t l = 1; l < P->blev.size(); ++l) {
        BatchLevel& F = P->blev[l - 1];
        BatchLevel& C = P->blev[l];
        CKE(launch_restrict_plain_batch(C.d_geom_fine, C.d_geom, C.d_cells, C.ncells, F.delta, C.delta, s));
        CKE(launch_restrict_ghosts_batch(C.d_geom_fine, C.d_geom, C.d_store, C.nstore_items, F.phi[0], C.phi[0],
                                         C.phi[1], C.phiold, s));
    }
    if (P->mixed) {
        for (auto& L : P->blev) CKE(launch_cast_all(L.phi[0], L.pt, L.pool, s));
        return bcast(P);
    }
    return bnorms(P);
}

hipError_t batch_outputs(Plan* P, double* phi) {
    BatchLevel& B = P->blev[0];
    return launch_copy_out_batch(B.d_geom, P->d_uoff, B.d_cells, B.ncells, P->mixed ? B.phi[0] : B.phi[B.cur], phi,
                                 P->stream);
}

hipError_t batch_smooth_finest(Plan* P) { return P->mixed ? bsmooth_corr(P, 0) : bsmooth(P, 0); }

hipError_t batch_smooth_level(Plan* P, int l) { return P->mixed ? bsmooth_corr(P, l) : bsmooth(P, l); }

int batch_parity(const Plan* P) { return P->blev.empty() ? 0 : P->blev[0].cur; }

void batch_flip_parity(Plan* P) {
    if (!P->blev.empty()) P->blev[0].cur ^= 1;
}

}  // namespace vmg
