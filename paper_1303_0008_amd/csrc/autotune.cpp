// Autotuner: picks the fused-sweep tile height and z-chunk of a plan's finest
// level by timing the real smoother kernel on the plan's own buffers (HIP
// events on the plan's stream).  Results are cached per (grid shape, precision,
// boundary kind, batch size) in the process and, if the environment variable
// VMG_TUNE_CACHE names a file, in that file ("key ty zc us" lines).
#include <hip/hip_runtime.h>

#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <string>

#include "vmg_internal.h"
#include "vmg_plan.h"

namespace vmg {

namespace {
std::mutex g_tune_mu;
std::map<std::string, SmoothCfg> g_tune_cache;

std::string tune_key(const Plan* P) {
    char buf[160];
    const Geom& g = P->grids[0].lev[0].g;
    std::snprintf(buf, sizeof(buf), "gfx950:%dx%dx%d:%s:%s:%d", g.n0, g.n1, g.n2, P->mixed ? "mixed" : "fp64",
                  P->periodic ? "per" : "dir", (int)P->grids.size());
    return buf;
}

void load_file_cache() {
    const char* path = std::getenv("VMG_TUNE_CACHE");
    if (!path) return;
    FILE* f = std::fopen(path, "r");
    if (!f) return;
    char key[160];
    int ty, zc;
    double us;
    while (std::fscanf(f, "%159s %d %d %lf", key, &ty, &zc, &us) == 4) {
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

// one finest-level sweep of the plan (every grid), alternating buffers
hipError_t sweep_once(Plan* P) {
    if (P->batched) return batch_smooth_finest(P);
    for (auto& G : P->grids) {
        hipError_t e = P->mixed ? smooth_corr_level(P, G, 0) : smooth_level_public(P, G, 0);
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}
}  // namespace

vmg_status autotune(Plan* P) {
    const std::string key = tune_key(P);
    {
        std::lock_guard<std::mutex> lk(g_tune_mu);
        if (g_tune_cache.empty()) load_file_cache();
        auto it = g_tune_cache.find(key);
        if (it != g_tune_cache.end()) {
            P->cfg = it->second;
            P->tuned_from_cache = true;
            return P->batched && batch_build_smooth_items(P) != hipSuccess ? fail(VMG_EHIP, "items") : VMG_OK;
        }
    }
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)
        return fail(VMG_EHIP, "hipEventCreate failed");
    const int tys[3] = {8, 4, 16}, zcs[3] = {16, 8, 32};
    SmoothCfg best = P->cfg;
    double best_us = 1e300;
    const int64_t cu = P->cell_updates, fs = P->finest_sweeps;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) {
            SmoothCfg c;
            c.ty = tys[a];
            c.zc = zcs[b];
            P->cfg = c;
            if (P->batched && batch_build_smooth_items(P) != hipSuccess) return fail(VMG_EHIP, "items");
            const int warm = 2, reps = 6;
            bool ok = true;
            for (int r = 0; r < warm && ok; ++r) ok = sweep_once(P) == hipSuccess;
            ok = ok && hipEventRecord(e0, P->stream) == hipSuccess;
            for (int r = 0; r < reps && ok; ++r) ok = sweep_once(P) == hipSuccess;
            ok = ok && hipEventRecord(e1, P->stream) == hipSuccess && hipEventSynchronize(e1) == hipSuccess;
            float ms = 0.0f;
            if (!ok || hipEventElapsedTime(&ms, e0, e1) != hipSuccess) {
                (void)hipEventDestroy(e0);
                (void)hipEventDestroy(e1);
                return fail(VMG_EHIP, "autotune timing failed");
            }
            const double us = 1e3 * ms / reps;
            P->tune_log.push_back({c, us});
            if (us < best_us) {
                best_us = us;
                best = c;
            }
        }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    P->cfg = best;
    P->cell_updates = cu;
    P->finest_sweeps = fs;
    if (P->batched && batch_build_smooth_items(P) != hipSuccess) return fail(VMG_EHIP, "items");
    // the sweeps above ran on zero-filled buffers and toggled the ping-pong
    // state; every solve resets it, so nothing else needs restoring
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    append_file_cache(key, best, best_us);
    return VMG_OK;
}

}  // namespace vmg
