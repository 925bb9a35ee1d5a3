// Autotuner: picks the fused sweep's tile height and z chunk for every level of
// a plan by timing the real smoother kernel on the plan's own buffers (HIP
// events on the plan's stream).  The finest level tries heights {8,4,16,12} x
// chunks {16,8,32}; each coarser level heights {8,4,16,12} x chunks {16,8,4,2},
// since short chunks spread small grids over the chip.  Results are cached per
// (grid shape, precision, boundary kind, batch size, level) in the process and,
// if the environment variable VMG_TUNE_CACHE names a file, in that file
// ("key ty zc us" lines).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "vmg_internal.h"
#include "vmg_plan.h"

namespace vmg {

namespace {
std::mutex g_tune_mu;
std::map<std::string, SmoothCfg> g_tune_cache;
bool g_file_loaded = false;

std::string tune_key(const Plan* P, int l) {
    char buf[192];
    const Geom& g = P->grids[0].lev[0].g;
    std::snprintf(buf, sizeof(buf), "gfx950:%dx%dx%d:%s:%s:%d:L%d", g.n0, g.n1, g.n2, P->mixed ? "mixed" : "fp64",
                  P->periodic ? "per" : "dir", (int)P->grids.size(), l);
    return buf;
}

void load_file_cache() {
    g_file_loaded = true;
    const char* path = std::getenv("VMG_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[192];
    int ty, zc;
    double us;
    while (std::fscanf(f, "%191s %d %d %lf", key, &ty, &zc, &us) == 4) {
        SmoothCfg c;
        c.ty = ty;
        c.zc = zc;
        g_tune_cache[key] = c;
    }
    std::fclose(f);
}

void append_file_cache(const std::string& key, const SmoothCfg& c, double us) {
    const char* path = std::getenv("VMG_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "a");
    if (!f) return;
    std::fprintf(f, "%s %d %d %.3f\n", key.c_str(), c.ty, c.zc, us);
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
    append_file_cache(key, c, us);
}

// Install schedule c on level l.
hipError_t apply(Plan* P, int l, const SmoothCfg& c) {
    if (l == 0) P->cfg = c;
    if (P->batched) return batch_set_level_cfg(P, l, c);
    if (l > 0) P->lcfg[l] = c;
    return hipSuccess;
}

// One sweep of level l (every grid of the plan).
hipError_t sweep_level(Plan* P, int l) {
    if (P->batched) return batch_smooth_level(P, l);
    for (auto& G : P->grids) {
        hipError_t e = P->mixed ? smooth_corr_level(P, G, l) : smooth_level_public(P, G, l);
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
        if (cached(key, best)) {
            P->tuned_from_cache = true;
            if (apply(P, l, best) != hipSuccess) st = fail(VMG_EHIP, "autotune: work list upload failed");
            continue;
        }
        std::vector<SmoothCfg> cands;
        const int tys[4] = {8, 4, 16, 12};
        const int zf[3] = {16, 8, 32}, zcoarse[4] = {16, 8, 4, 2};
        for (int a = 0; a < 4; ++a) {
            if (l == 0)
                for (int b = 0; b < 3; ++b) cands.push_back(SmoothCfg{tys[a], zf[b]});
            else
                for (int b = 0; b < 4; ++b) cands.push_back(SmoothCfg{tys[a], zcoarse[b]});
        }
        double best_us = 1e300;
        for (const SmoothCfg& c : cands) {
            const int warm = 2, reps = 6;
            bool ok = apply(P, l, c) == hipSuccess;
            for (int r = 0; r < warm && ok; ++r) ok = sweep_level(P, l) == hipSuccess;
            ok = ok && hipEventRecord(e0, P->stream) == hipSuccess;
            for (int r = 0; r < reps && ok; ++r) ok = sweep_level(P, l) == hipSuccess;
            ok = ok && hipEventRecord(e1, P->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                st = fail(VMG_EHIP, "autotune timing failed");
                break;
            }
            const double us = 1e3 * ms / reps;
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

}  // namespace vmg
