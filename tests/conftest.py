import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)


def pytest_configure(config):
    config.addinivalue_line("markers", "gpu: needs an MI355X (gfx950) GPU")
    config.addinivalue_line("markers", "slow: CPU test that takes more than ~20 s")


@pytest.fixture(scope="session")
def oracle_mod():
    from oracle import oracle as O
    O.lib()
    return O


TUNE_FILE = os.path.join(ROOT, "paper_1303_0008_amd", "tune_gfx950.txt")


def bench_schedules(prec_name, n=256):
    """Per-level sweep schedules {level: (tile_y, z_chunk, pipe)} of the committed
    tuning file for the periodic n^3 plan of one precision ("fp64" or "mixed")
    -- the schedules the benchmark replays."""
    out = {}
    with open(TUNE_FILE) as f:
        for line in f:
            parts = line.split()
            key = parts[0].split(":") if parts else []
            if len(key) != 6 or not key[5].startswith("L") or len(parts) not in (4, 5):
                continue
            if key[1] == f"{n}x{n}x{n}" and key[2] == prec_name and key[3] == "per" and key[4] == "1":
                pipe = int(parts[3]) if len(parts) == 5 else 0
                out[int(key[5][1:])] = (int(parts[1]), int(parts[2]), pipe)
    return out


def bench_cycle(prec_name, n=256):
    """Cycle schedule of the committed tuning file for the periodic n^3 plan, or None."""
    with open(TUNE_FILE) as f:
        for line in f:
            parts = line.split()
            if parts and parts[0] == f"gfx950:{n}x{n}x{n}:{prec_name}:per:1:cycle" and len(parts) in (8, 10):
                v = [int(x) for x in parts[1:-1]] + [0, 0]
                return dict(zip(("nu1", "nu2", "inner_cycles", "coarse_sweeps", "coarse_tail", "batch_blocks",
                                 "coarse_nu1", "coarse_nu2"), v))
    return None


def install_schedules(plan, schedules, cycle=None):
    """Install {level: (tile_y, z_chunk, pipe)} on the levels the plan sweeps, and
    a cycle schedule if given (before the sweep schedules: the coarse tail
    decides which levels are swept)."""
    if cycle is not None:
        plan.set_cycle(**cycle)
    for lev, (ty, zc, pipe) in sorted(schedules.items()):
        if lev < plan.level_count():
            plan.set_schedule(lev, ty, zc, pipe)


def residual_fields(V, torch, oracle_mod, delta, d_t, phi_t, alpha, kappa):
    """Residual field of phi on the GPU (vmg_residual) and from the oracle, cell by
    cell on a periodic unit box.  Returns (max |d_gpu - d_oracle|, bound, max
    |d_oracle|, gpu result, oracle info).  The bound is what rounding allows
    two evaluations of the same definition in different order: each term of d
    is at most 12 |phi|_inf / h^2 or |Q| (the root, below kappa |delta|_inf +
    |cbar|), each side rounds a few dozen times, so 64 eps times their sum."""
    n2, n1, n0 = delta.shape
    h = 1.0 / n0
    d_gpu = torch.empty_like(phi_t)
    with V.Plan([V.make_grid((n0, n1, n2))], V.make_params(alpha, kappa, 1e-8)) as p:
        r = p.residual(0, d_t, phi_t, d=d_gpu)
    phi = phi_t.cpu().numpy()
    dg = d_gpu.cpu().numpy()
    del d_gpu
    d_or, info = oracle_mod.residual(delta, phi, alpha, kappa)
    eps = np.finfo(np.float64).eps
    bound = 64 * eps * (12 * np.abs(phi).max() / h ** 2 + abs(kappa) * np.abs(delta).max() + abs(info["cbar"]) + 1)
    err = float(np.abs(dg - d_or).max())
    dmax = float(np.abs(d_or).max())
    del dg, d_or
    return err, float(bound), dmax, r, info
