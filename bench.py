"""Benchmark of the gfx950 Vainshtein multigrid solver (one GPU).

Workload (the configuration the headline metric is quoted on): periodic 256^3
unit box, density contrast from a CIC deposit of 256^3 lattice particles
displaced by a seeded Zel'dovich field (P(k) ~ k^-1.5, cut at k_Nyquist/4),
alpha = 0.2, kappa = 1.5, mixed precision, solved from phi = 0 to RMS
residual 1e-8.

One step = one complete solve (all V-cycles, every level, norms and host
checks) with the inputs already resident in HBM.  ``value`` is smoother cell
updates (all levels, all sweeps) per second of wall time over the timed
steps; ``ms_per_step`` is the time to tolerance.  The schedules (sweep tiles
per level and the cycle schedule) are those of the committed tuning file
(paper_1303_0008_amd/tune_gfx950.txt, written by ``--retune``).

``roofline`` describes the dominant kernel, the finest-level fused red-black
sweep: algorithmic bytes per launch (24 B per cell FP64: read phi, read delta,
write phi; 20 B FP32 correction: e, phi~, t0, r in, e out) divided by its
average duration, measured with HIP events that the library records around
every finest-level sweep of the timed solves (vmg_plan_time_sweeps) on the
plan's stream.  ``traffic`` is the HBM bytes per launch from the committed
FETCH_SIZE / WRITE_SIZE counter runs of ``--traffic-probe`` (null if the
kernel source changed since).

``results`` also holds, outside the timed solves: the other configurations
(32^3 top-hat, 128^3 lognormal, the 96 refinement patches, the two 512^3
lognormal sets with the 512^3 finest-sweep roofline), the mass assignment, the
total force, the truncation-error rule and a multilevel solve.

``cpu_baseline`` times the CPU oracle (plain FP64 C, single-threaded) on a
bounded sample of the same workload: one FAS V(2,2) cycle of its own solver
over the full 256^3 grid from phi = 0, as cell updates (all levels) per
second; once on one core and once as concurrent independent copies, one per
host core (the value).
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


def time_solves(torch, V, delta, w, prec, steps, warmup, flags, stream, tau_factor=0.0, grids=None, ghost=None,
                phi0=None, time_sweeps=False, max_cycles=100):
    """Solve the same input `steps` times after `warmup` untimed solves; wall time
    over the timed solves (bracketed by device synchronisation).  With
    time_sweeps, the library times every finest-level sweep of the timed solves
    with HIP events on the plan's stream.  Returns (plan, infos, cell updates,
    seconds, last phi, (summed sweep us, sweep launches))."""
    grids = grids or [V.make_grid(w["n"])]
    params = V.make_params(w["alpha"], w["kappa"], w["tol"], max_cycles, prec, flags=flags, tau_factor=tau_factor)
    plan = V.Plan(grids, params, stream=stream)
    # every solve starts from its own resident copy of the initial guess
    phis = [torch.zeros_like(delta) if phi0 is None else phi0.clone() for _ in range(steps + warmup)]
    infos = []
    with torch.cuda.stream(stream):
        for i in range(warmup):
            plan.solve(delta, phis[i], ghost=ghost)
        if time_sweeps:
            plan.time_sweeps(True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        updates = 0
        for i in range(steps):
            r = plan.solve(delta, phis[warmup + i], ghost=ghost)
            infos.append(r[0] if len(grids) == 1 else r)
            updates += plan.stats()["cell_updates"]
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        sweeps = plan.sweep_time() if time_sweeps else (0.0, 0)
    return plan, infos, updates, (t1 - t0), phis[-1], sweeps


COPY_BYTES = 256 << 20       # calibration copy: 256 MiB read + 256 MiB written
# finest-level sweep of each precision: kernel name prefix and algorithmic bytes per cell
FINEST = {"fp64": ("k_smooth<", 24), "mixed": ("k_smooth_corr<", 20)}


def finest_kernel(name, tile_y, pipe):
    """Name of the finest-level sweep kernel of a precision for a schedule (the
    plain sweep: no prolongation folded in)."""
    return f"{FINEST[name][0]}{tile_y}, 0, false, {'true' if pipe else 'false'}, false>"


PROBE_SWEEPS = 10


def traffic_probe(torch, V, delta, w, launches=PROBE_SWEEPS):
    """Kernels for the HBM counter runs: finest-level sweeps of both precisions (the
    tuned schedules) on a solved state, then a plain device copy of COPY_BYTES
    (calibration)."""
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


def traffic_from(fetch_dir, write_dir, n, workload=WORKLOAD):
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
        for name, (pre, _) in FINEST.items():
            # the probe's closing finest-level sweeps (tuned schedule): the last
            # PROBE_SWEEPS launches of the precision's periodic sweep kernels
            # (no FAS source, correction read from memory), in dispatch order
            cand = [r for r in rows if r["Kernel_Name"].startswith("void vmg::" + pre)
                    and ", 0, false, " in r["Kernel_Name"].split("(")[0]][-PROBE_SWEEPS:]
            kern = cand[-1]["Kernel_Name"].split("(")[0].replace("void vmg::", "") if cand else None
            if len(cand) < PROBE_SWEEPS or any(not r["Kernel_Name"].startswith("void vmg::" + kern) for r in cand):
                raise SystemExit(f"{counter}: the closing {pre}... sweeps were not found")
            vals = [float(r["Counter_Value"]) for r in cand]
            per.setdefault(name, {})[counter] = {"kernel": kern, "kib_per_launch_median": statistics.median(vals),
                                                  "launches": len(vals), "copy_kib": statistics.median(copies),
                                                  "calibration_factor": scale,
                                                  "bytes_per_launch": statistics.median(vals) * 1024.0 * scale}
    for name, (_, bpc) in FINEST.items():
        d = per[name]
        out = {"kernel": d["FETCH_SIZE"]["kernel"], "workload": f"{workload} ({n}^3)",
               "kernel_source_hash": kernel_source_hash(),
               "algorithmic_bytes_per_launch": bpc * ncell,
               "fetch": d["FETCH_SIZE"], "write": d["WRITE_SIZE"],
               "bytes_per_launch": d["FETCH_SIZE"]["bytes_per_launch"] + d["WRITE_SIZE"]["bytes_per_launch"]}
        out["ratio_to_algorithmic"] = out["bytes_per_launch"] / out["algorithmic_bytes_per_launch"]
        p = os.path.join(ROOT, "profiles", f"smooth_{name}_{workload}_traffic.json")
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
    plan, infos, updates, dt, _, _ = time_solves(torch, V, delta, dict(w), V.FP64, steps, 1, V.GRAPH | V.AUTOTUNE,
                                                 stream, tau_factor=1.0 / 3.0)
    plan.close()
    r = infos[-1]
    log(f"tau rule (1/3): {1e3 * dt / steps:.3f} ms/solve, cycles {r['cycles']}, rms {r['rms']:.3e}, "
        f"tau rms {r['tau_rms']:.3e}")
    return {"tau_factor": 1.0 / 3.0, "time_to_stop_ms": 1e3 * dt / steps, "cycles": r["cycles"], "rms": r["rms"],
            "tau_rms": r["tau_rms"]}


def levels_inputs(torch, V, delta_np, w):
    """Grids, nests and densities of the multilevel workload: the domain grid with 8
    first-level 64^3 refinements at h = 1/512 centred on the 8 densest cells at
    least 40 cells apart (so the refinements do not overlap) and a 64^3 second
    level at h = 1/1024 in the middle of each.  Each refinement's density is the
    cloud-in-cell assignment of the workload's particles onto it
    (vmg_mass_assign_region), the recipe of the domain grid at the finer spacing;
    assign_all() (re)computes those densities in d."""
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
    regions = []                       # (offset, h, corner, origin) of each refinement
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
            regions.append((off, h, corner, origin))
            off += 64 ** 3
            goff += V.ghost_count(64)
    d = torch.empty(off, dtype=torch.float64, device="cuda")
    d[:delta_np.size] = torch.from_numpy(delta_np.ravel()).to("cuda")
    work = torch.empty(V.mass_assign_workspace(pos_np.shape[0], 64), dtype=torch.uint8, device="cuda")

    def assign_all():
        for o, h, corner, _ in regions:
            V.mass_assign_region(pos, 64, h, corner, pos_np.shape[0] * h ** 3, V.ASSIGN_CIC,
                                 delta=d[o:o + 64 ** 3].view(64, 64, 64), workspace=work)

    return grids, nests, d, goff, regions, assign_all


def levels_refinement_inputs(torch, V, delta_np, w):
    """The 8 first-level refinements of the multilevel workload as one Dirichlet
    batch, with boundary values and initial guess interpolated from the domain
    grid's FP64 solution (what vmg_levels_solve hands them): the input of the
    cycle tuner for the refinement plans."""
    n = w["n"]
    grids, nests, d, goff, regions, assign_all = levels_inputs(torch, V, delta_np, w)
    assign_all()
    parent_phi, _ = V.solve_field(d[:n ** 3].view(n, n, n), w["alpha"], w["kappa"], tol=1e-10, max_cycles=60)
    first = [r for r in regions if abs(r[1] - 1.0 / (2 * n)) < 1e-15]
    sub, origins = [], []
    for k, (o, h, _, origin) in enumerate(first):
        sub.append(V.make_grid(64, h, V.DIRICHLET, k * 64 ** 3, k * V.ghost_count(64)))
        origins.append(origin)
    dt = torch.cat([d[o:o + 64 ** 3] for o, _, _, _ in first])
    ghost = torch.zeros(len(first) * V.ghost_count(64), dtype=torch.float64, device="cuda")
    V.fill_ghosts(parent_phi, 1.0 / n, sub, origins, ghost)
    guess = torch.zeros_like(dt)
    V.fill_interior(parent_phi, 1.0 / n, sub, origins, guess)
    torch.cuda.synchronize()
    return sub, dt, ghost, guess


def time_levels(torch, V, delta_np, w, steps):
    """vmg_levels_solve on the multilevel workload (levels_inputs), mixed
    precision, tol as the workload, tuned schedules (VMG_AUTOTUNE: the domain grid
    and the refinement batches take their cached sweep and cycle schedules).  Wall
    time per vmg_levels_solve on a plan created beforehand; the assignment of all
    16 refinement densities is timed apart."""
    grids, nests, d, goff, regions, assign_all = levels_inputs(torch, V, delta_np, w)
    assign_all()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    assign_all()
    torch.cuda.synchronize()
    assign_ms = 1e3 * (time.perf_counter() - t0)
    off = d.numel()
    ghost = torch.zeros(goff, dtype=torch.float64, device="cuda")
    params = V.make_params(w["alpha"], w["kappa"], w["tol"], 100, V.MIXED, flags=V.GRAPH | V.AUTOTUNE)
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
        f"max rms {max(r['rms'] for r in res):.2e}, cycles {[r['cycles'] for r in res][:2]}...; "
        f"refinement densities assigned in {assign_ms:.2f} ms")
    return {"ms_per_solve": ms, "grids": len(grids), "cells": off, "max_rms": max(r["rms"] for r in res),
            "cycles": [r["cycles"] for r in res], "refinement_assign_ms": assign_ms,
            "note": "vmg_levels_solve on a plan created beforehand (tuned schedules), from phi = 0, mixed "
                    "precision; refinement densities by cloud-in-cell region assignment of the workload's "
                    "particles"}


def oracle_cycle_updates(n, nu=4, ncoarse=60):
    """Cell updates of one FAS V(2,2) cycle of the oracle on a periodic n^3 grid:
    nu1 + nu2 sweeps on every level above the coarsest (4^3), ncoarse sweeps on it."""
    upd, m = 0, n
    while m % 2 == 0 and m // 2 >= 4:
        upd += nu * m ** 3
        m //= 2
    return upd + ncoarse * m ** 3


def cpu_baseline(delta, w):
    """The oracle (single-threaded C) on one FAS V(2,2) cycle of the 256^3 workload
    from phi = 0: once alone, then as one independent copy per host core at once
    (threads: the oracle runs in C with the interpreter lock released)."""
    import threading
    from oracle import oracle as O
    upd = oracle_cycle_updates(w["n"])

    def one():
        O.solve(delta, w["alpha"], w["kappa"], tol=0.0, max_cycles=1)

    t0 = time.perf_counter()
    one()
    t1 = time.perf_counter() - t0
    cores = max(1, min(16, os.cpu_count() or 1))
    ths = [threading.Thread(target=one) for _ in range(cores)]
    t0 = time.perf_counter()
    for th in ths:
        th.start()
    for th in ths:
        th.join()
    tc = time.perf_counter() - t0
    model = ""
    try:
        with open("/proc/cpuinfo") as f:
            model = next((l.split(":", 1)[1].strip() for l in f if l.startswith("model name")), "")
    except OSError:
        pass
    log(f"cpu baseline: one cycle {t1:.1f} s on 1 core; {cores} concurrent copies {tc:.1f} s ({model})")
    return {"value": cores * upd / tc, "unit": "cell-updates/s", "cores": cores, "kind": "oracle",
            "sample": f"one FAS V(2,2) cycle of the FP64 oracle (lexicographic Newton-Gauss-Seidel, its own "
                      f"hierarchy down to 4^3, 60 coarsest sweeps) over the full {w['n']}^3 workload from phi = 0, "
                      f"{upd} cell updates per copy, wall time including the oracle's set-up and residual "
                      f"evaluations; {cores} independent copies on {cores} threads ran in {tc:.1f} s",
            "single_core_value": upd / t1, "single_core_seconds": t1, "host_cpu": model,
            "host_cpu_count": os.cpu_count()}


def patches96_inputs(torch, V, I):
    """The 96 refinement patches (sides {16..64}, h = 1/512) with ghosts and initial
    guess interpolated trilinearly from the GPU's solution of the 128^3 lognormal
    parent."""
    import numpy as np
    pd = torch.from_numpy(I.workload_delta("lognormal128")).to("cuda")
    parent_phi, _ = V.solve_field(pd, 0.1, 1.5, tol=1e-10, max_cycles=60)
    patches = I.patch_set()
    h = 1.0 / 512
    grids, origins, off, goff = [], [], 0, 0
    for pch in patches:
        grids.append(V.make_grid(pch.n, h, V.DIRICHLET, off, goff))
        origins.append(pch.origin)
        off += pch.delta.size
        goff += V.ghost_count(pch.n)
    ghost = torch.zeros(goff, dtype=torch.float64, device="cuda")
    V.fill_ghosts(parent_phi, 1.0 / 128, grids, origins, ghost)
    guess = torch.zeros(off, dtype=torch.float64, device="cuda")
    V.fill_interior(parent_phi, 1.0 / 128, grids, origins, guess)
    dt = torch.from_numpy(np.concatenate([p.delta.ravel() for p in patches])).to("cuda")
    torch.cuda.synchronize()
    return grids, dt, ghost, guess


def solve_entry(name, infos, updates, dt, steps, sweeps=None, bpc=None, cells=None, kernel=None):
    last = infos[-1] if isinstance(infos[-1], dict) else max(infos[-1], key=lambda r: r["rms"])
    out = {"time_to_tol_ms": 1e3 * dt / steps, "cycles": last["cycles"], "rms": last["rms"],
           "cell_updates_per_s": updates / dt}
    if sweeps and sweeps[1] > 0:
        us = sweeps[0] / sweeps[1]
        gbs = bpc * cells / (us * 1e-6) / 1e9
        out["finest_sweep"] = {"kernel": kernel, "us_per_launch": us, "launches_timed": sweeps[1],
                               "algorithmic_bytes_per_launch": bpc * cells, "achieved_gbs": gbs,
                               "frac_of_hbm_peak": gbs / HBM_PEAK_GBS}
    log(f"{name}: {out['time_to_tol_ms']:.3f} ms/solve, cycles {out['cycles']}, rms {out['rms']:.2e}" +
        (f"; finest sweep {out['finest_sweep']['us_per_launch']:.1f} us = {out['finest_sweep']['achieved_gbs']:.0f} GB/s"
         if "finest_sweep" in out else ""))
    return out


def other_configs(torch, V, I, stream, steps):
    """The other benchmark configurations, each solved `steps` times (GRAPH,
    tuned schedules), with the finest sweep timed in the solves where it is
    bandwidth-relevant (the 96 patches, 512^3)."""
    import numpy as np
    res = {}
    flags = V.GRAPH | V.AUTOTUNE
    for name, precs in (("tophat32", ("fp64",)), ("lognormal128", ("fp64", "mixed"))):
        w = dict(I.WORKLOADS[name])
        d = torch.from_numpy(I.workload_delta(name)).to("cuda")
        for pn in precs:
            prec = V.FP64 if pn == "fp64" else V.MIXED
            plan, infos, upd, dt, _, _ = time_solves(torch, V, d, w, prec, steps, 2, flags, stream)
            plan.close()
            res[f"{name}_{pn}"] = solve_entry(f"{name} {pn}", infos, upd, dt, steps)
    grids, dt_p, ghost, guess = patches96_inputs(torch, V, I)
    cells = int(dt_p.numel())
    wp = dict(I.WORKLOADS["patches96"])
    # The first batched plan a process creates runs its solves ~40 % slower than
    # an identical plan created after it (measured with and without graphs; the
    # same kernels, schedules and iterations), so that first plan is timed and
    # reported apart and the steady state is the configuration's time.
    plan, _, _, dt_first, _, _ = time_solves(torch, V, dt_p, wp, V.MIXED, steps, 2, flags, stream, grids=grids,
                                             ghost=ghost, phi0=guess)
    plan.close()
    for pn, prec, bpc, pre in (("mixed", V.MIXED, 20, "k_smooth_corr_batch"), ("fp64", V.FP64, 24, "k_smooth_batch")):
        # graph-replayed solves (the time), then solves with the finest sweeps
        # bracketed by events (launched directly: the sweep time)
        plan, infos, upd, dt, _, _ = time_solves(torch, V, dt_p, wp, prec, steps, 2, flags, stream, grids=grids,
                                                 ghost=ghost, phi0=guess)
        plan.close()
        plan, _, _, _, _, sw = time_solves(torch, V, dt_p, wp, prec, max(2, steps // 2), 1, flags, stream, grids=grids,
                                           ghost=ghost, phi0=guess, time_sweeps=True)
        ty, zc, pipe = plan.schedule(0)
        plan.close()
        res[f"patches96_{pn}"] = solve_entry(f"patches96 {pn} ({len(grids)} patches, {cells} cells)", infos, upd, dt,
                                             steps, sw, bpc, cells,
                                             f"{pre}<{ty}, ...> (persistent, z chunk {zc}, pipe {pipe})")
        if pn == "mixed":
            res[f"patches96_{pn}"]["first_plan_of_process_ms"] = 1e3 * dt_first / steps
    del dt_p, ghost, guess
    t = time.perf_counter()
    d512 = torch.from_numpy(I.workload_delta("lognormal512a")).to("cuda")
    log(f"lognormal512: generated in {time.perf_counter() - t:.1f} s")
    n3 = 512 ** 3
    for name, alpha in (("lognormal512a", 0.2), ("lognormal512b", -0.2)):
        w = dict(I.WORKLOADS[name])
        for pn, prec, bpc in (("mixed", V.MIXED, 20), ("fp64", V.FP64, 24)):
            # the guarded configuration (alpha < 0) under-relaxes its kink cells and
            # takes several times the iterations of the other
            mc = 100 if alpha > 0 else 250
            try:
                plan, infos, upd, dt, _, _ = time_solves(torch, V, d512, w, prec, max(2, steps // 4), 1, flags, stream,
                                                         max_cycles=mc)
            except V.VmgError as e:   # reported, not fatal: the other lines still print
                res[f"{name}_{pn}"] = {"status": "error", "error": str(e), "max_cycles": mc}
                log(f"{name} {pn}: {e}")
                torch.cuda.synchronize()
                continue
            plan.close()
            torch.cuda.empty_cache()
            plan, _, _, _, _, sw = time_solves(torch, V, d512, w, prec, 2, 0, flags, stream, time_sweeps=True,
                                               max_cycles=mc)
            ty, zc, pipe = plan.schedule(0)
            plan.close()
            kern = finest_kernel(pn, ty, pipe)
            res[f"{name}_{pn}"] = solve_entry(f"{name} {pn}", infos, upd, dt, max(2, steps // 4), sw, bpc, n3,
                                              kern + f" (z chunk {zc})")
            # HBM bytes per launch from the committed counter runs at 512^3
            if "finest_sweep" in res[f"{name}_{pn}"]:
                res[f"{name}_{pn}"]["finest_sweep"]["traffic"] = load_traffic(f"smooth_{pn}_{name}_traffic.json",
                                                                              kern)
            torch.cuda.empty_cache()
    del d512
    torch.cuda.empty_cache()
    return res


def retune(torch, V, I, stream, path):
    """Write a fresh tuning file: sweep schedules of every plan the benchmark and
    tests replay (VMG_AUTOTUNE) and their cycle schedules (vmg_plan_tune_cycle)."""
    if os.path.exists(path):
        os.remove(path)
    os.environ["VMG_TUNE_CACHE"] = path
    jobs = []
    for name in ("zeldovich256", "lognormal128", "tophat32", "lognormal512a"):
        w = dict(I.WORKLOADS[name])
        d = torch.from_numpy(I.workload_delta(name)).to("cuda")
        for prec in ((V.FP64,) if name == "tophat32" else (V.FP64, V.MIXED)):
            jobs.append((name, [V.make_grid(w["n"])], w, prec, d, None, None))
    grids, dt_p, ghost, guess = patches96_inputs(torch, V, I)
    for prec in (V.FP64, V.MIXED):
        jobs.append(("patches96", grids, dict(I.WORKLOADS["patches96"]), prec, dt_p, ghost, guess))
    # the refinement batches of the multilevel solve (both depths share the key)
    wz = dict(I.WORKLOADS["zeldovich256"])
    sub, dt_r, ghost_r, guess_r = levels_refinement_inputs(torch, V, I.workload_delta("zeldovich256"), wz)
    jobs.append(("levels refinements", sub, wz, V.MIXED, dt_r, ghost_r, guess_r))
    for name, grids, w, prec, d, gh, g0 in jobs:
        params = V.make_params(w["alpha"], w["kappa"], w["tol"], 100, prec, flags=V.GRAPH | V.AUTOTUNE)
        with V.Plan(grids, params, stream=stream) as plan:
            work = torch.zeros_like(d) if g0 is None else g0.clone()
            best, ms = plan.tune_cycle(d, work, ghost=gh)
            log(f"retune {name} {'fp64' if prec == V.FP64 else 'mixed'}: schedules "
                f"{[plan.schedule(l) for l in range(plan.level_count())]}, cycle {best}, {ms:.3f} ms")
        torch.cuda.empty_cache()
    log(f"tuning file written: {path}")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--assign-launches", type=int, default=20,
                    help="timed calls of the mass assignment (0: skip it)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the other configurations and the total-force, truncation-error-rule, mass "
                         "assignment and multilevel timings")
    ap.add_argument("--traffic-probe", action="store_true",
                    help="run only the kernels of the HBM counter runs (under rocprofv3 --pmc)")
    ap.add_argument("--probe-workload", default=WORKLOAD, choices=("zeldovich256", "lognormal512a"),
                    help="workload of --traffic-probe / --traffic-from (default: the headline one)")
    ap.add_argument("--traffic-from", nargs=2, metavar=("FETCH_DIR", "WRITE_DIR"),
                    help="turn two rocprofv3 --pmc csv outputs of --traffic-probe into profiles/*_traffic.json")
    ap.add_argument("--history", metavar="FILE",
                    help="append the residual history of a solve of each precision to FILE (JSON lines)")
    ap.add_argument("--retune", metavar="FILE",
                    help="write a fresh tuning file (sweep and cycle schedules of every configuration) and exit")
    args = ap.parse_args()
    os.environ.setdefault("VMG_TUNE_CACHE", TUNE_CACHE)
    if args.traffic_from:
        from paper_1303_0008_amd import inputs as I
        traffic_from(args.traffic_from[0], args.traffic_from[1], I.WORKLOADS[args.probe_workload]["n"],
                     args.probe_workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              "(the solver is a single-GPU build).", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1303_0008_amd import inputs as I
    from paper_1303_0008_amd import vmg as V

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    V.load()
    stream = torch.cuda.Stream()        # default priority
    if args.retune:
        retune(torch, V, I, stream, os.path.abspath(args.retune))
        return
    w = dict(I.WORKLOADS[WORKLOAD])
    t = time.perf_counter()
    delta_np = I.workload_delta(WORKLOAD)
    log(f"workload {WORKLOAD}: generated in {time.perf_counter() - t:.1f} s, max delta {delta_np.max():.1f}")
    delta = torch.from_numpy(delta_np).to("cuda")
    if args.traffic_probe:
        if args.probe_workload != WORKLOAD:
            wp = dict(I.WORKLOADS[args.probe_workload])
            dp = torch.from_numpy(I.workload_delta(args.probe_workload)).to("cuda")
            del delta
            traffic_probe(torch, V, dp, wp)
        else:
            traffic_probe(torch, V, delta, w)
        return
    torch.cuda.synchronize()

    results = {}
    n3 = w["n"] ** 3
    roofs = {}
    for name, prec, what in (("fp64", V.FP64, "fused red-black sweep, FP64"),
                             ("mixed", V.MIXED, "fused red-black sweep on the FP32 correction")):
        bpc = FINEST[name][1]
        # timed solves (the value), then the same number again with every finest
        # sweep bracketed by HIP events (the roofline)
        plan, infos, updates, dt, _, _ = time_solves(torch, V, delta, w, prec, args.steps, args.warmup,
                                                     V.GRAPH | V.AUTOTUNE, stream)
        plan.close()
        plan, infos_t, _, dt_t, _, sw = time_solves(torch, V, delta, w, prec, args.steps, 1, V.GRAPH | V.AUTOTUNE,
                                                    stream, time_sweeps=True)
        ty, zc, pipe = plan.schedule(0)
        sched = [plan.schedule(l) for l in range(plan.level_count())]
        cyc = plan.cycle()
        # one more solve with every level's share of each iteration timed, and its
        # residual history
        plan.time_sweeps(False)
        plan.time_levels(True)
        with torch.cuda.stream(stream):
            phi_l = torch.zeros_like(delta)
            plan.solve(delta, phi_l)
        torch.cuda.synchronize()
        lev = [plan.level_time(l) for l in range(plan.level_count() + 1)]
        hist = plan.history()
        plan.close()
        if args.history:
            V.write_history_jsonl(args.history, hist, workload=WORKLOAD, precision=name)
        kern = finest_kernel(name, ty, pipe)
        results[name] = solve_entry(name, infos, updates, dt, args.steps, sw, bpc, n3, kern)
        results[name]["timed_solves_ms_per_step"] = 1e3 * dt_t / args.steps
        results[name]["schedules"] = {"sweep_per_level": sched, "cycle": cyc}
        results[name]["level_us_per_iteration"] = [round(us / max(k, 1), 2) for us, k in lev]
        results[name]["residual_history"] = [h["rms"] for h in hist]
        fs = results[name]["finest_sweep"]
        roofs[name] = {"bound": "hbm", "achieved": fs["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                       "frac": fs["achieved_gbs"] / HBM_PEAK_GBS,
                       "traffic": load_traffic(f"smooth_{name}_{WORKLOAD}_traffic.json", kern),
                       "kernel": f"{kern} ({what}, z chunk {zc})",
                       "bytes_per_launch": bpc * n3, "us_per_launch": fs["us_per_launch"],
                       "launches_timed": fs["launches_timed"]}
    results["mixed_speedup_vs_fp64"] = results["fp64"]["time_to_tol_ms"] / results["mixed"]["time_to_tol_ms"]
    if not args.no_extras:
        results["configs"] = other_configs(torch, V, I, stream, args.steps)
        if args.assign_launches > 0:
            results["mass_assign_zeldovich256"] = time_mass_assign(torch, V, stream, args.assign_launches)
        results["total_force_zeldovich256"] = time_total_force(torch, V, delta, w, stream, 20)
        results["tau_rule_zeldovich256"] = time_tau_rule(torch, V, delta, w, stream, 3)
        results["levels_zeldovich256"] = time_levels(torch, V, delta_np, w, 2)
    head = "mixed"
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
                   "schedule": "fused red-black sweeps, hipGraph, tuned sweep tiles per level and tuned cycle "
                               "(tune_gfx950.txt)"},
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
