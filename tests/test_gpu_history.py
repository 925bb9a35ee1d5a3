"""Residual history and per-level timing of a solve (the measurement hooks).

vmg_plan_history returns the norms of the initial guess and after every
iteration: its first entry is the result's rms0, its last the result's rms, and
its length the iteration count plus one; every entry is pinned to the FP64
residual the oracle computes of the same iterate at the end.  vmg_plan_time_levels
times each level's share of later iterations: every level that a V-cycle visits
gets a positive time, the pieces sum to no more than the solve's wall time, and
the timed (directly launched) solve gives the same iterate as the graph replay.
"""
import json
import time

import numpy as np
import pytest

from paper_1303_0008_amd import inputs as I

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


@pytest.fixture(scope="module")
def V():
    from paper_1303_0008_amd import vmg
    vmg.load()
    return vmg


def say(*a):
    print(*a, flush=True)


@pytest.mark.parametrize("prec_name", ["fp64", "mixed"])
def test_history_and_level_times(torch_cuda, V, oracle_mod, prec_name, tmp_path):
    torch = torch_cuda
    prec = V.FP64 if prec_name == "fp64" else V.MIXED
    n = 64
    delta = I.lognormal((n, n, n), 611, sigma=1.2)
    d_t = torch.from_numpy(delta).cuda()
    say(f"history/level timing: {prec_name}, periodic {n}^3")
    params = V.make_params(0.2, 1.5, 1e-9, 60, prec, flags=V.GRAPH)
    with V.Plan([V.make_grid(n)], params) as plan:
        phi_g = torch.zeros_like(d_t)
        info = plan.solve(d_t, phi_g)[0]
        hist = plan.history()
        assert len(hist) == info["cycles"] + 1
        assert hist[0]["rms"] == pytest.approx(info["rms0"], rel=1e-12)
        assert hist[-1]["rms"] == pytest.approx(info["rms"], rel=1e-12)
        assert hist[-1]["rms"] <= 1e-9 < hist[0]["rms"]
        assert all(h["n_guarded"] >= 0 for h in hist)
        # the last entry is the FP64 residual of the returned iterate (the oracle's)
        _, ref = oracle_mod.residual(delta, phi_g.cpu().numpy(), 0.2, 1.5, want_field=False)
        assert hist[-1]["rms"] == pytest.approx(ref["rms"], rel=1e-6, abs=1e-13)
        path = tmp_path / "history.jsonl"
        V.write_history_jsonl(str(path), hist, precision=prec_name, n=n)
        lines = [json.loads(l) for l in path.read_text().splitlines()]
        assert [l["iteration"] for l in lines] == list(range(len(hist)))
        assert lines[-1]["rms"] == hist[-1]["rms"] and lines[0]["precision"] == prec_name

        # per-level timing: the same iterate, launched directly
        nlev = plan.level_count() + 1
        plan.time_levels(True)
        phi_t = torch.zeros_like(d_t)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        info_t = plan.solve(d_t, phi_t)[0]
        torch.cuda.synchronize()
        wall_us = 1e6 * (time.perf_counter() - t0)
        assert info_t["cycles"] == info["cycles"]
        assert torch.equal(phi_t, phi_g)
        times = [plan.level_time(l) for l in range(nlev)]
        say("  level times (us, iterations):", [(round(u, 1), k) for u, k in times])
        assert all(k == info["cycles"] for _, k in times)
        # level 0 and every swept level below it have work in every iteration
        for l in range(plan.level_count()):
            assert times[l][0] > 0.0, l
        assert sum(u for u, _ in times) < wall_us
        plan.time_levels(False)
        phi_r = torch.zeros_like(d_t)
        plan.solve(d_t, phi_r)
        assert torch.equal(phi_r, phi_g)
        with pytest.raises(V.VmgError):
            plan.level_time(nlev + 3)
