// Autotuner (Sec. V of the paper: the code "needs more tunings").  Two parts:
//
//  * Sweep schedules, at plan creation (VMG_AUTOTUNE): for every level that
//    runs the fused sweep, time the real smoother kernel on the plan's own
//    buffers (HIP events on the plan's stream), two sweeps at a time, for tile
//    heights {8,4,16,12} x z chunks ({16,8,32,64} on the finest level,
//    {16,8,4,2} below, since short chunks spread small grids over the chip) x
//    both pipeline shapes, plus the brick schedule (without the z march: two
//    sweeps per launch on the coarser levels of a periodic plan, one on every
//    level of a Dirichlet batch), and keep the fastest.
//  * The cycle schedule, on request (vmg_plan_tune_cycle): time complete
//    solves of a given input (from the caller's initial guess) to the plan's
//    tolerance for candidate nu1/nu2,
//    inner cycles, coarsest sweeps, coarse tail and persistent launch size, by
//    coordinate search, and keep the fastest.
//
// Results are cached per (grid shape, precision, boundary kind, batch size,
// level or "cycle") in the process and, if the environment variable
// VMG_TUNE_CACHE names a file, in that file: one line per key, "key values...
// time" (sweep: tile height, z chunk, pipeline shape, microseconds per sweep;
// cycle: nu1, nu2, inner cycles, coarsest sweeps, tail, launch size,
// milliseconds per solve).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <map>
#include <mutex>
#include <sstream>
#include <string>
#include <vector>

#include "vmg_internal.h"
#include "vmg_plan.h"

namespace vmg {

namespace {
std::mutex g_tune_mu;
std::map<std::string, SmoothCfg> g_tune_cache;
std::map<std::string, vmg_cycle> g_cycle_cache;
bool g_file_loaded = false;

std::string plan_key(const Plan* P) {
    char buf[192];
    const Geom& g = P->grids[0].lev[0].g;
    std::snprintf(buf, sizeof(buf), "gfx950:%dx%dx%d:%s:%s:%d", g.n0, g.n1, g.n2, P->mixed ? "mixed" : "fp64",
                  P->periodic ? "per" : "dir", (int)P->grids.size());
    return buf;
}

std::string tune_key(const Plan* P, int l) { return plan_key(P) + ":L" + std::to_string(l); }
std::string cycle_key(const Plan* P) { return plan_key(P) + ":cycle"; }

// Lines: "key ty zc us" (pipeline shape 0), "key ty zc pipe us",
// "key:cycle nu1 nu2 inner coarse tail blocks ms" (coarse levels as the finest) or
// "key:cycle nu1 nu2 inner coarse tail blocks coarse_nu1 coarse_nu2 ms".
void load_file_cache() {
    g_file_loaded = true;
    const char* path = std::getenv("VMG_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char line[512];
    while (std::fgets(line, sizeof(line), f)) {
        std::istringstream in(line);
        std::string key;
        if (!(in >> key)) continue;
        std::vector<double> v;
        double x;
        while (in >> x) v.push_back(x);
        const bool cyc = key.size() > 6 && key.compare(key.size() - 6, 6, ":cycle") == 0;
        if (cyc && (v.size() == 7 || v.size() == 9)) {
            vmg_cycle c;
            c.nu1 = (int)v[0]; c.nu2 = (int)v[1]; c.inner_cycles = (int)v[2];
            c.coarse_sweeps = (int)v[3]; c.coarse_tail = (int)v[4]; c.batch_blocks = (int)v[5];
            c.coarse_nu1 = v.size() == 9 ? (int)v[6] : 0;
            c.coarse_nu2 = v.size() == 9 ? (int)v[7] : 0;
            g_cycle_cache[key] = c;
        } else if (!cyc && (v.size() == 3 || v.size() == 4)) {
            SmoothCfg c;
            c.ty = (int)v[0];
            c.zc = (int)v[1];
            c.pipe = v.size() == 4 ? (int)v[2] : 0;
            // only schedules vmg_plan_set_schedule would accept (others are re-tuned)
            const bool ok = (c.ty == 4 || c.ty == 8 || c.ty == 12 || c.ty == 16) && c.zc >= 2 && c.zc <= 1024 &&
                            (c.zc & 1) == 0 && c.pipe >= 0 && c.pipe <= PIPE_BRICK;
            if (ok) g_tune_cache[key] = c;
        }
    }
    std::fclose(f);
}

void append_line(const std::string& line) {
    const char* path = std::getenv("VMG_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s\n", line.c_str());
    std::fclose(f);
}

bool cached(const std::string& key, SmoothCfg& c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_file_loaded) load_file_cache();
    auto it = g_tune_cache.find(key);
    if (it == g_tune_cache.end()) return false;
    c = it->second;
    return true;
}

void remember(const std::string& key, const SmoothCfg& c, double us) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = c;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s %d %d %d %.3f", key.c_str(), c.ty, c.zc, c.pipe, us);
    append_line(buf);
}

void remember_cycle(const std::string& key, const vmg_cycle& c, double ms) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_cycle_cache[key] = c;
    char buf[256];
    std::snprintf(buf, sizeof(buf), "%s %d %d %d %d %d %d %d %d %.3f", key.c_str(), c.nu1, c.nu2, c.inner_cycles,
                  c.coarse_sweeps, c.coarse_tail, c.batch_blocks, c.coarse_nu1, c.coarse_nu2, ms);
    append_line(buf);
}

// Install schedule c on level l.
hipError_t apply(Plan* P, int l, const SmoothCfg& c) {
    if (l == 0) P->cfg = c;
    if (P->batched) return batch_set_level_cfg(P, l, c);
    if (l > 0) P->lcfg[l] = c;
    return hipSuccess;
}

// n pre-sweeps of level l (every grid of the plan), then, with post, the coarse
// correction's prolongation and n post-sweeps, as a V-cycle issues them.
hipError_t sweep_level(Plan* P, int l, int n, bool post = false) {
    if (P->batched) {
        for (int s = 0; s < (post ? 2 * n : n); ++s) {
            hipError_t e = batch_smooth_level(P, l);
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    for (auto& G : P->grids) {
        hipError_t e = P->mixed ? smooth_corr_level_n(P, G, l, n) : smooth_level_public(P, G, l, n);
        if (e == hipSuccess && post && l + 1 < (int)G.lev.size())
            e = P->mixed ? post_smooth_corr(P, G, l, n) : post_smooth(P, G, l, n);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

// Levels of the plan that run the fused sweep: every level above the coarsest,
// except those the periodic coarse tail handles in one launch.
int swept_level_count(const Plan* P) {
    if (P->batched) {
        int n = 0;
        for (size_t l = 0; l < P->blev.size(); ++l)
            if (P->blev[l].nsitems > 0) n = (int)l + 1;
        return n;
    }
    const int tl = tail_level(P, P->grids[0]);
    return tl > 0 ? tl : (int)P->grids[0].lev.size() - 1;
}

bool cached_cycle(const Plan* P, vmg_cycle* c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    if (!g_file_loaded) load_file_cache();
    auto it = g_cycle_cache.find(cycle_key(P));
    if (it == g_cycle_cache.end()) return false;
    *c = it->second;
    return true;
}

// Sweep schedules of every swept level (plan creation, VMG_AUTOTUNE).
vmg_status autotune(Plan* P) {
    if (!P->batched) P->lcfg.assign(P->grids[0].lev.size(), SmoothCfg{0, 0});
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(VMG_EHIP, "hipEventCreate failed");
    const int64_t cu = P->cell_updates, fs = P->finest_sweeps;
    const int nlev = swept_level_count(P);
    vmg_status st = VMG_OK;
    for (int l = 0; l < nlev && st == VMG_OK; ++l) {
        const std::string key = tune_key(P, l);
        SmoothCfg best;
        // the brick schedule runs on the coarser levels of periodic plans and on
        // every level of Dirichlet batches
        if (cached(key, best) && (best.pipe != PIPE_BRICK || l > 0 || P->batched)) {
            P->tuned_from_cache = true;
            if (apply(P, l, best) != hipSuccess) st = fail(VMG_EHIP, "autotune: work list upload failed");
            continue;
        }
        std::vector<SmoothCfg> cands;
        const int tys[4] = {8, 4, 16, 12};
        const int zf[4] = {16, 8, 32, 64}, zcoarse[4] = {16, 8, 4, 2};
        for (int pipe = 1; pipe >= 0; --pipe)
            for (int a = 0; a < 4; ++a) {
                if (l == 0)
                    for (int b = 0; b < 4; ++b) cands.push_back(SmoothCfg{tys[a], zf[b], pipe});
                else
                    for (int b = 0; b < 4; ++b) cands.push_back(SmoothCfg{tys[a], zcoarse[b], pipe});
            }
        // coarser periodic levels may also run their sweeps in pairs on bricks, and
        // Dirichlet batches one at a time on every level
        if (l > 0 || P->batched) cands.push_back(SmoothCfg{8, 8, PIPE_BRICK});
        double best_us = 1e300;
        // the finest level: plain sweeps; below it, a V(2,2) cycle's smoothing (two
        // sweeps, the coarse correction, two sweeps) per repetition
        const bool post = l > 0;
        const int per_rep = post ? 4 : 2;
        for (const SmoothCfg& c : cands) {
            const int warm = 2, reps = 6;
            bool ok = apply(P, l, c) == hipSuccess;
            for (int r = 0; r < warm && ok; ++r) ok = sweep_level(P, l, 2, post) == hipSuccess;
            ok = ok && hipEventRecord(e0, P->stream) == hipSuccess;
            for (int r = 0; r < reps && ok; ++r) ok = sweep_level(P, l, 2, post) == hipSuccess;
            ok = ok && hipEventRecord(e1, P->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(VMG_EHIP, "autotune timing failed");
                break;
            }
            const double us = 1e3 * ms / (per_rep * reps);
            P->tune_log.push_back({l, c, us});
            if (us < best_us) {
                best_us = us;
                best = c;
            }
        }
        if (st != VMG_OK) break;
        if (apply(P, l, best) != hipSuccess) {
            st = fail(VMG_EHIP, "autotune: work list upload failed");
            break;
        }
        remember(key, best, best_us);
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    // the timing sweeps ran on the plan's zero-filled buffers and toggled their
    // ping-pong state; every solve resets both, so only the counters need restoring
    P->cell_updates = cu;
    P->finest_sweeps = fs;
    return st;
}

// Cycle schedule by coordinate search over complete solves (vmg_plan_tune_cycle).
vmg_status tune_cycle(Plan* P, const double* delta, const double* ghost, const double* source, double* phi_work,
                      vmg_cycle* best_out, double* best_ms_out) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(VMG_EHIP, "hipEventCreate failed");
    int64_t nphi = 0;
    for (const auto& G : P->grids)
        nphi = std::max<int64_t>(nphi, G.desc.offset + (int64_t)G.desc.n[0] * G.desc.n[1] * G.desc.n[2]);
    // every trial starts from the initial guess phi_work holds on entry
    double* guess = nullptr;
    if (hipMalloc((void**)&guess, sizeof(double) * (size_t)nphi) != hipSuccess) {
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(VMG_ENOMEM, "tune_cycle: hipMalloc failed");
    }
    if (hipMemcpyAsync(guess, phi_work, sizeof(double) * (size_t)nphi, hipMemcpyDeviceToDevice, P->stream) !=
        hipSuccess) {
        (void)hipFree(guess);
        (void)hipEventDestroy(e0);
        (void)hipEventDestroy(e1);
        return fail(VMG_EHIP, "tune_cycle: copy of the initial guess failed");
    }
    // median of three solves; < 0 when the candidate does not converge
    auto time_solve = [&](double& ms_out) -> vmg_status {
        std::vector<double> ts;
        std::vector<vmg_result> res(P->grids.size());
        for (int r = 0; r < 3; ++r) {
            if (hipMemcpyAsync(phi_work, guess, sizeof(double) * (size_t)nphi, hipMemcpyDeviceToDevice, P->stream) !=
                hipSuccess)
                return fail(VMG_EHIP, "tune_cycle: copy of the initial guess failed");
            if (hipEventRecord(e0, P->stream) != hipSuccess) return fail(VMG_EHIP, "event record failed");
            const vmg_status st = solve(P, delta, ghost, source, phi_work, res.data());
            if (st == VMG_ENOCONV || st == VMG_ENONFINITE) {
                ms_out = -1.0;
                return VMG_OK;
            }
            if (st != VMG_OK) return st;
            float ms = 0.0f;
            if (hipEventRecord(e1, P->stream) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
                hipEventElapsedTime(&ms, e0, e1) != hipSuccess)
                return fail(VMG_EHIP, "event timing failed");
            ts.push_back(ms);
        }
        std::sort(ts.begin(), ts.end());
        ms_out = ts[1];
        return VMG_OK;
    };
    vmg_cycle best;
    get_cycle(P, &best);
    double best_ms = -1.0;
    vmg_status st = time_solve(best_ms);
    auto consider = [&](const vmg_cycle& c) -> vmg_status {
        vmg_status s2 = set_cycle(P, &c);
        if (s2 != VMG_OK) return s2;
        double ms = -1.0;
        if ((s2 = time_solve(ms)) != VMG_OK) return s2;
        if (ms > 0.0 && (best_ms < 0.0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
        }
        return VMG_OK;
    };
    const int nus[7][2] = {{1, 1}, {1, 2}, {2, 1}, {2, 2}, {2, 3}, {3, 2}, {3, 3}};
    for (int i = 0; i < 7 && st == VMG_OK; ++i) {
        vmg_cycle c = best;
        c.nu1 = nus[i][0];
        c.nu2 = nus[i][1];
        if (c.nu1 != best.nu1 || c.nu2 != best.nu2) st = consider(c);
    }
    // sweeps below the finest level: as the finest, or fewer
    const int cnus[4][2] = {{0, 0}, {1, 1}, {1, 2}, {2, 1}};
    for (int i = 0; i < 4 && st == VMG_OK; ++i) {
        vmg_cycle c = best;
        c.coarse_nu1 = cnus[i][0];
        c.coarse_nu2 = cnus[i][1];
        if (c.coarse_nu1 != best.coarse_nu1 || c.coarse_nu2 != best.coarse_nu2) st = consider(c);
    }
    if (P->mixed) {
        // inner cycles per outer step trade outer passes against inner work: more
        // of them can save a whole outer step; then the sweep counts once more
        for (int k = 1; k <= 6 && st == VMG_OK; ++k) {
            vmg_cycle c = best;
            c.inner_cycles = k;
            if (k != best.inner_cycles) st = consider(c);
        }
        for (int i = 0; i < 7 && st == VMG_OK; ++i) {
            vmg_cycle c = best;
            c.nu1 = nus[i][0];
            c.nu2 = nus[i][1];
            if (c.nu1 != best.nu1 || c.nu2 != best.nu2) st = consider(c);
        }
    }
    const int coarse[4] = {2, 4, 8, 16};
    for (int i = 0; i < 4 && st == VMG_OK; ++i) {
        vmg_cycle c = best;
        c.coarse_sweeps = coarse[i];
        if (c.coarse_sweeps != best.coarse_sweeps) st = consider(c);
    }
    if (P->periodic) {
        vmg_cycle c = best;
        c.coarse_tail = 1 - best.coarse_tail;
        if (st == VMG_OK) st = consider(c);
    } else {
        const int blocks[3] = {512, 1024, 2048};
        for (int i = 0; i < 3 && st == VMG_OK; ++i) {
            vmg_cycle c = best;
            c.batch_blocks = blocks[i];
            if (c.batch_blocks != best.batch_blocks) st = consider(c);
        }
    }
    (void)hipStreamSynchronize(P->stream);
    (void)hipFree(guess);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (st != VMG_OK) return st;
    if (best_ms < 0.0) return fail(VMG_ENOCONV, "tune_cycle: no candidate reached the tolerance");
    if ((st = set_cycle(P, &best)) != VMG_OK) return st;
    remember_cycle(cycle_key(P), best, best_ms);
    if (best_out) *best_out = best;
    if (best_ms_out) *best_ms_out = best_ms;
    return VMG_OK;
}

}  // namespace vmg
