"""Benchmark of the gfx950 Vainshtein multigrid solver (one GPU).

Workload (the configuration the headline metric is quoted on): periodic 256^3
unit box, density contrast from a CIC deposit of 256^3 lattice particles
displaced by a seeded Zel'dovich field (P(k) ~ k^-1.5, cut at k_Nyquist/4),
alpha = 0.2, kappa = 1.5, solved from phi = 0 to RMS residual 1e-8.

One step = one complete solve (all V-cycles, every level, norms and host
checks) with the inputs already resident in HBM.  ``value`` is smoother cell
updates (all levels, all sweeps) per second of wall time over the timed
steps; ``ms_per_step`` is the time to tolerance.

``roofline`` describes the dominant kernel, the finest-level fused red-black
sweep: algorithmic bytes per launch (24 B per cell: read phi, read delta,
write phi) divided by its average duration, timed here with HIP events around
back-to-back launches on the plan's stream.

``results.mass_assign_zeldovich256`` times the mass assignment (triangular-
shaped cloud and cloud in cell) of the workload's 256^3 particles onto the
256^3 grid, outside the solve.

``results`` also holds, each outside the timed solves: the total potential and
force kernel at 256^3 (bandwidth in algorithmic bytes), FP64 solves stopped by
the truncation-error rule (|d| <= |tau|/3), and a multilevel solve of the
workload with two nested levels of refinements.

``cpu_baseline`` times the CPU oracle (plain FP64 C, one thread) on a bounded
sample of the same workload: five lexicographic Newton-Gauss-Seidel sweeps
over the full 256^3 grid.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
WORKLOAD = "zeldovich256"
# Schedules the autotuner chose on MI355X for this workload (tile height and z chunk
# per level); the library re-tunes any plan whose key is missing from the file.
TUNE_CACHE = os.path.join(ROOT, "paper_1303_0008_amd", "tune_gfx950.txt")


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    h = hashlib.sha256()
    for f in ("device_common.h", "brick.h", "kernels.hip", "kernels_mixed.hip"):
        p = os.path.join(ROOT, "paper_1303_0008_amd", "csrc", f)
        if os.path.exists(p):
            h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def load_traffic(name, kernel):
    """HBM bytes per launch from committed rocprofv3 counter runs, if they were
    taken on the current kernel source and the same instantiation; otherwise None."""
    p = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(p):
        return None
    try:
        d = json.load(open(p))
    except Exception:
        return None
    if d.get("kernel_source_hash") != kernel_source_hash() or d.get("kernel") != kernel:
        return None
    return d.get("bytes_per_launch")


def time_solves(torch, V, delta, w, prec, steps, warmup, flags, stream, tau_factor=0.0):
    n = w["n"]
    params = V.make_params(w["alpha"], w["kappa"], w["tol"], 100, prec, flags=flags, tau_factor=tau_factor)
    plan = V.Plan([V.make_grid(n)], params, stream=stream)
    phis = [torch.zeros_like(delta) for _ in range(steps + warmup)]
    infos = []
    with torch.cuda.stream(stream):
        for i in range(warmup):
            plan.solve(delta, phis[i])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        updates = 0
        for i in range(steps):
            infos.append(plan.solve(delta, phis[warmup + i])[0])
            updates += plan.stats()["cell_updates"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
    return plan, infos, updates, (t1 - t0), phis[-1]


def time_smoother(torch, plan, stream, launches):
    """Average duration of the finest-level smoother, from HIP events on the plan's stream."""
    plan.smooth(2)                      # warm
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    plan.smooth(launches)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / launches


COPY_BYTES = 256 << 20       # calibration copy: 256 MiB read + 256 MiB written
# finest-level sweep of each precision: kernel name prefix / suffix (the tile height
# between them is the autotuner's choice) and algorithmic bytes per cell
FINEST = {"fp64": ("k_smooth<", ", 0, false>", 24), "mixed": ("k_smooth_corr<", ", 0, false>", 20)}


def finest_kernel(name, tile_y):
    pre, post, _ = FINEST[name]
    return f"{pre}{tile_y}{post}"


PROBE_SWEEPS = 10


def traffic_probe(torch, V, delta, w, launches=PROBE_SWEEPS):
    """Kernels for the HBM counter runs: finest-level sweeps of both precisions on
    a solved state, then a plain device copy of COPY_BYTES (calibration)."""
    stream = torch.cuda.Stream()
    for prec in (V.FP64, V.MIXED):
        plan = V.Plan([V.make_grid(w["n"])],
                      V.make_params(w["alpha"], w["kappa"], w["tol"], 100, prec, flags=V.AUTOTUNE), stream=stream)
        phi = torch.zeros_like(delta)
        with torch.cuda.stream(stream):
            plan.solve(delta, phi)
            plan.smooth(launches)
        torch.cuda.synchronize()
        plan.close()
    src = torch.ones(COPY_BYTES // 8, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    log(f"traffic probe done: {launches} sweeps per precision, 3 copies of {COPY_BYTES >> 20} MiB")


def _counter_rows(path):
    import csv
    import glob
    files = glob.glob(os.path.join(path, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise SystemExit(f"no counter_collection.csv under {path}")
    rows = []
    for f in files:
        with open(f) as fh:
            rows.extend(csv.DictReader(fh))
    return rows


def traffic_from(fetch_dir, write_dir, n):
    """Per-launch HBM bytes of the finest sweeps from a FETCH_SIZE run and a
    WRITE_SIZE run of --traffic-probe, each scaled so that the calibration copy
    reads / writes exactly COPY_BYTES; writes the JSON files the roofline reads."""
    import statistics
    ncell = n ** 3
    per = {}
    for counter, path in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        rows = [r for r in _counter_rows(path) if r.get("Counter_Name") == counter]
        rows.sort(key=lambda r: int(r["Dispatch_Id"]))
        tail = rows[-3:]      # the probe ends with the three calibration copies
        if len(tail) < 3 or not all("copy" in r["Kernel_Name"].lower() for r in tail):
            raise SystemExit(f"{counter}: calibration copies not found at the end of the run")
        copies = [float(r["Counter_Value"]) for r in tail]
        # counter KiB -> bytes, times the factor that makes the copy read/write COPY_BYTES
        scale = COPY_BYTES / (1024.0 * statistics.median(copies))
        for name, (pre, post, _) in FINEST.items():
            # the probe's closing finest-level sweeps (tuned schedule): the last
            # PROBE_SWEEPS launches of the precision's sweep kernels, in dispatch order
            cand = [r for r in rows if r["Kernel_Name"].startswith("void vmg::" + pre)
                    and r["Kernel_Name"].split("(")[0].endswith(post)][-PROBE_SWEEPS:]
            kern = cand[-1]["Kernel_Name"].split("(")[0].replace("void vmg::", "") if cand else None
            if len(cand) < PROBE_SWEEPS or any(not r["Kernel_Name"].startswith("void vmg::" + kern) for r in cand):
                raise SystemExit(f"{counter}: the closing {pre}..{post} sweeps were not found")
            vals = [float(r["Counter_Value"]) for r in cand]
            per.setdefault(name, {})[counter] = {"kernel": kern, "kib_per_launch_median": statistics.median(vals),
                                                  "launches": len(vals), "copy_kib": statistics.median(copies),
                                                  "calibration_factor": scale,
                                                  "bytes_per_launch": statistics.median(vals) * 1024.0 * scale}
    for name, (_, _, bpc) in FINEST.items():
        d = per[name]
        out = {"kernel": d["FETCH_SIZE"]["kernel"], "workload": f"{WORKLOAD} ({n}^3)",
               "kernel_source_hash": kernel_source_hash(),
               "algorithmic_bytes_per_launch": bpc * ncell,
               "fetch": d["FETCH_SIZE"], "write": d["WRITE_SIZE"],
               "bytes_per_launch": d["FETCH_SIZE"]["bytes_per_launch"] + d["WRITE_SIZE"]["bytes_per_launch"]}
        out["ratio_to_algorithmic"] = out["bytes_per_launch"] / out["algorithmic_bytes_per_launch"]
        p = os.path.join(ROOT, "profiles", f"smooth_{name}_{WORKLOAD}_traffic.json")
        with open(p, "w") as fh:
            json.dump(out, fh, indent=1)
        log(f"{name}: {out['bytes_per_launch'] / 1e6:.1f} MB per launch "
            f"({out['ratio_to_algorithmic']:.2f} x algorithmic) -> {p}")


def time_mass_assign(torch, V, stream, launches):
    """Mass assignment of the workload's particles (256^3 lattice particles after
    the Zel'dovich displacement) with both schemes: average duration per call from
    HIP events on `stream` (each call = binning by brick, LDS accumulation and the
    outer-layer passes)."""
    from paper_1303_0008_amd import inputs as I
    pos_np = I.zeldovich_particles(256, I.BASE_SEED + 3, I.ZELDOVICH_AMPLITUDE)
    pos = torch.from_numpy(pos_np).to("cuda")
    delta = torch.empty((256, 256, 256), dtype=torch.float64, device="cuda")
    work = torch.empty(V.mass_assign_workspace(pos_np.shape[0], 256), dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    out = {}
    for name, scheme, m in (("tsc", V.ASSIGN_TSC, 27), ("cic", V.ASSIGN_CIC, 8)):
        V.mass_assign(pos, 256, scheme, delta=delta, workspace=work, stream=stream)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(launches):
            V.mass_assign(pos, 256, scheme, delta=delta, workspace=work, stream=stream)
        e1.record(stream)
        e1.synchronize()
        ms = e0.elapsed_time(e1) / launches
        npart = pos_np.shape[0]
        out[name] = {"ms_per_call": ms, "particles_per_s": npart / (ms * 1e-3),
                     "atomics_per_s": npart * m / (ms * 1e-3), "particles": npart, "grid": 256}
        log(f"mass assignment {name}: {ms * 1e3:.1f} us per call, {npart / (ms * 1e-3) / 1e9:.2f} G particles/s")
    return out


def time_total_force(torch, V, delta, w, stream, launches):
    """Total potential and force (vmg_total_force) on the workload's 256^3 grid from
    the solved brane-bending mode and the Newtonian potential (alpha = 0 solve of
    the same density, kappa = (3/2) Omega_m a with Omega_m = 0.257, a = 1)."""
    n = w["n"]
    phi, _ = V.solve_field(delta, w["alpha"], w["kappa"], tol=w["tol"])
    phin, _ = V.solve_field(delta, 0.0, 1.5 * 0.257, tol=w["tol"])
    psi = torch.empty_like(phi)
    force = torch.empty((3,) + tuple(phi.shape), dtype=torch.float64, device="cuda")
    V.total_force(phin, phi, 1.0 / n, psi=psi, force=force, stream=stream)
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(launches):
        V.total_force(phin, phi, 1.0 / n, psi=psi, force=force, stream=stream)
    e1.record(stream)
    e1.synchronize()
    us = 1e3 * e0.elapsed_time(e1) / launches
    bpc = 48                                   # phi_N, phi in; Psi and three force components out
    gbs = bpc * n ** 3 / (us * 1e-6) / 1e9
    log(f"total force: {us:.1f} us per call = {gbs:.0f} GB/s algorithmic")
    return {"us_per_call": us, "algorithmic_bytes_per_cell": bpc, "achieved_gbs": gbs,
            "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}


def time_tau_rule(torch, V, delta, w, stream, steps):
    """FP64 solves that also stop on the truncation-error rule |d| <= |tau|/3."""
    plan, infos, updates, dt, _ = time_solves(torch, V, delta, dict(w), V.FP64, steps, 1, V.GRAPH | V.AUTOTUNE,
                                              stream, tau_factor=1.0 / 3.0)
    plan.close()
    r = infos[-1]
    log(f"tau rule (1/3): {1e3 * dt / steps:.3f} ms/solve, cycles {r['cycles']}, rms {r['rms']:.3e}, "
        f"tau rms {r['tau_rms']:.3e}")
    return {"tau_factor": 1.0 / 3.0, "time_to_stop_ms": 1e3 * dt / steps, "cycles": r["cycles"], "rms": r["rms"],
            "tau_rms": r["tau_rms"]}


def time_levels(torch, V, delta_np, w, steps):
    """vmg_levels_solve on the workload's domain grid with 8 first-level 64^3
    refinements at h = 1/512 centred on the 8 densest cells at least 40 cells
    apart (so the refinements do not overlap) and a 64^3 second level at
    h = 1/1024 in the middle of each (mixed precision, tol as the workload).
    Each refinement's density is the cloud-in-cell assignment of the
    workload's particles onto it (vmg_mass_assign_region), the recipe of the
    domain grid at the finer spacing.  Wall time per vmg_levels_solve on a plan
    created beforehand; the assignment of all 16 refinements is timed apart."""
    import numpy as np
    from paper_1303_0008_amd import inputs as I
    n = w["n"]
    flat = np.argsort(delta_np.ravel())[::-1]
    peaks = []
    for f in flat:
        k, j, i = np.unravel_index(f, delta_np.shape)
        if all(max(min(abs(c - q), n - abs(c - q)) for c, q in zip((i, j, k), p)) >= 40 for p in peaks):
            peaks.append((i, j, k))
        if len(peaks) == 8:
            break
    pos_np = I.zeldovich_particles(n, I.BASE_SEED + 3, I.ZELDOVICH_AMPLITUDE)
    pos = torch.from_numpy(pos_np).to("cuda")
    grids = [V.make_grid(n)]
    nests = [V.make_nest(-1)]
    regions = []                       # (offset, h, corner) of each refinement
    off, goff = delta_np.size, 0
    corners = {}
    for lev, h in ((1, 1.0 / (2 * n)), (2, 1.0 / (4 * n))):
        for t, p in enumerate(peaks):
            parent = 0 if lev == 1 else 1 + t
            origin = tuple((2 * c - 32) % (2 * n) for c in p) if lev == 1 else (32, 32, 32)
            base = (0.0, 0.0, 0.0) if lev == 1 else corners[parent]
            corner = tuple((base[a] + origin[a] * h) % 1.0 for a in range(3))
            corners[len(grids)] = corner
            grids.append(V.make_grid(64, h, V.DIRICHLET, off, goff))
            nests.append(V.make_nest(parent, origin))
            regions.append((off, h, corner))
            off += 64 ** 3
            goff += V.ghost_count(64)
    d = torch.empty(off, dtype=torch.float64, device="cuda")
    d[:delta_np.size] = torch.from_numpy(delta_np.ravel()).to("cuda")
    work = torch.empty(V.mass_assign_workspace(pos_np.shape[0], 64), dtype=torch.uint8, device="cuda")

    def assign_all():
        for o, h, corner in regions:
            V.mass_assign_region(pos, 64, h, corner, pos_np.shape[0] * h ** 3, V.ASSIGN_CIC,
                                 delta=d[o:o + 64 ** 3].view(64, 64, 64), workspace=work)

    assign_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assign_all()
    torch.cuda.synchronize()
    assign_ms = 1e3 * (time.perf_counter() - t0)
    ghost = torch.zeros(goff, dtype=torch.float64, device="cuda")
    params = V.make_params(w["alpha"], w["kappa"], w["tol"], 100, V.MIXED, flags=V.GRAPH)
    phis = [torch.zeros_like(d) for _ in range(steps + 1)]
    with V.LevelsPlan(grids, nests, params) as L:
        L.solve(d, ghost, phis[0])
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for k in range(steps):
            res = L.solve(d, ghost, phis[k + 1])
        torch.cuda.synchronize()
        ms = 1e3 * (time.perf_counter() - t0) / steps
    log(f"levels: {ms:.2f} ms per multilevel solve ({len(grids)} grids, {off} cells), "
        f"max rms {max(r['rms'] for r in res):.2e}; refinement densities assigned in {assign_ms:.2f} ms")
    return {"ms_per_solve": ms, "grids": len(grids), "cells": off, "max_rms": max(r["rms"] for r in res),
            "cycles": [r["cycles"] for r in res], "refinement_assign_ms": assign_ms,
            "note": "vmg_levels_solve on a plan created beforehand, from phi = 0, mixed precision; refinement "
                    "densities by cloud-in-cell region assignment of the workload's particles"}


def cpu_baseline(delta, w, sweeps=5):
    from oracle import oracle as O
    import numpy as np
    phi = np.zeros_like(delta)
    t0 = time.perf_counter()
    O.relax(delta, phi, w["alpha"], w["kappa"], sweeps)
    dt = time.perf_counter() - t0
    cells = delta.size * sweeps
    return {"value": cells / dt, "unit": "cell-updates/s", "cores": 1, "kind": "oracle",
            "sample": f"{sweeps} lexicographic Newton-Gauss-Seidel sweeps of the FP64 oracle over the full "
                      f"{w['n']}^3 workload from phi = 0 ({cells} cell updates, {dt:.1f} s, single thread)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--smooth-launches", type=int, default=50)
    ap.add_argument("--assign-launches", type=int, default=20,
                    help="timed calls of the mass assignment (0: skip it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the total-force, truncation-error-rule and multilevel timings")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only the kernels of the HBM counter runs (under rocprofv3 --pmc)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc csv outputs of --traffic-probe into profiles/*_traffic.json")
    args = ap.parse_args()
    os.environ.setdefault("VMG_TUNE_CACHE", TUNE_CACHE)
    if args.traffic_from:
        from paper_1303_0008_amd import inputs as I
        traffic_from(args.traffic_from[0], args.traffic_from[1], I.WORKLOADS[WORKLOAD]["n"])
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver is a single-GPU build).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_1303_0008_amd import inputs as I
    from paper_1303_0008_amd import vmg as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    V.load()
    w = dict(I.WORKLOADS[WORKLOAD])
    t = time.perf_counter()
    delta_np = I.workload_delta(WORKLOAD)
    log(f"workload {WORKLOAD}: generated in {time.perf_counter() - t:.1f} s, max delta {delta_np.max():.1f}")
    delta = torch.from_numpy(delta_np).to("cuda")
    if args.traffic_probe:
        traffic_probe(torch, V, delta, w)
        return
    stream = torch.cuda.Stream()        # default priority
    torch.cuda.synchronize()

    results = {}
    n3 = w["n"] ** 3
    roofs = {}
    for name, prec, bpc, what in (("fp64", V.FP64, 24, "fused red-black sweep, FP64"),
                                  ("mixed", V.MIXED, 20, "fused red-black sweep on the FP32 correction")):
        plan, infos, updates, dt, _ = time_solves(torch, V, delta, w, prec, args.steps, args.warmup,
                                                  V.GRAPH | V.AUTOTUNE, stream)
        sched = plan.config()
        ms = 1e3 * dt / args.steps
        smooth_ms = time_smoother(torch, plan, stream, args.smooth_launches)
        plan.close()
        achieved = bpc * n3 / (smooth_ms * 1e-3) / 1e9
        log(f"{name}: {ms:.3f} ms/solve, cycles {infos[-1]['cycles']}, rms {infos[-1]['rms']:.3e}; "
            f"smoother {smooth_ms * 1e3:.1f} us/launch = {achieved:.0f} GB/s, "
            f"{n3 / (smooth_ms * 1e-3) / 1e9:.1f} G cell-updates/s")
        results[name] = {"time_to_tol_ms": ms, "cycles": infos[-1]["cycles"], "rms": infos[-1]["rms"],
                         "cell_updates_per_s": updates / dt,
                         "smoother_us_per_launch": smooth_ms * 1e3,
                         "smoother_cell_updates_per_s": n3 / (smooth_ms * 1e-3),
                         "finest_schedule": {"tile_y": sched["tile_y"], "z_chunk": sched["z_chunk"]}}
        kern = finest_kernel(name, sched["tile_y"])
        roofs[name] = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": achieved / HBM_PEAK_GBS,
                       "traffic": load_traffic(f"smooth_{name}_zeldovich256_traffic.json", kern),
                       "kernel": f"{kern} ({what}, z chunk {sched['z_chunk']})",
                       "bytes_per_launch": bpc * n3, "us_per_launch": smooth_ms * 1e3}
    if args.assign_launches > 0:
        results["mass_assign_zeldovich256"] = time_mass_assign(torch, V, stream, args.assign_launches)
    if not args.no_extras:
        results["total_force_zeldovich256"] = time_total_force(torch, V, delta, w, stream, 20)
        results["tau_rule_zeldovich256"] = time_tau_rule(torch, V, delta, w, stream, 3)
        results["levels_zeldovich256"] = time_levels(torch, V, delta_np, w, 2)
    head = "mixed"
    results["mixed_speedup_vs_fp64"] = results["fp64"]["time_to_tol_ms"] / results["mixed"]["time_to_tol_ms"]
    roof = dict(roofs[head])
    roof["fp64_smoother"] = roofs["fp64"]

    line = {
        "metric": "cell-updates/s (smoother, all levels) over the solve to RMS residual 1e-8 at 256^3",
        "value": results[head]["cell_updates_per_s"],
        "unit": "cell-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": results[head]["time_to_tol_ms"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64",
        "data": "synthetic",
        "config": {"workload": "zeldovich256: periodic 256^3, Zel'dovich+CIC delta (P~k^-1.5, "
                               "cut k_Nyq/4), alpha=0.2, kappa=1.5, tol 1e-8, phi0=0",
                   "n": w["n"], "alpha": w["alpha"], "kappa": w["kappa"], "tol": w["tol"],
                   "precision": "mixed (FP32 correction V-cycle, FP64 defect correction)",
                   "schedule": "V(2,2) fused red-black, hipGraph, autotuned tiles per level"},
        "roofline": roof,
        "results": results,
    }
    if not args.no_cpu_baseline:
        log("cpu baseline (oracle) ...")
        line["cpu_baseline"] = cpu_baseline(delta_np, w)
    else:
        line["cpu_baseline"] = None
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
