"""Autotuner: the chosen schedule is one of the candidates and gives the same
answer as the default schedule (tile shape and z-chunk only change the blocking)."""
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


@pytest.mark.parametrize("prec", [0, 1])
def test_autotuned_plan_matches_default(torch_cuda, prec):
    torch = torch_cuda
    from paper_1303_0008_amd import vmg as V
    d = torch.from_numpy(I.lognormal(64, 801, sigma=1.0)).to("cuda")
    outs, cfgs = [], []
    for flags in (0, V.AUTOTUNE):
        phi = torch.zeros_like(d)
        with V.Plan([V.make_grid(64)], V.make_params(0.1, 1.5, 1e-11, 60, prec, flags=flags)) as p:
            cfgs.append(p.config())
            info = p.solve(d, phi)[0]
        outs.append((phi.cpu().numpy(), info))
    print(cfgs, flush=True)
    assert cfgs[1]["tile_y"] in (4, 8, 16) and cfgs[1]["z_chunk"] in (8, 16, 32)
    a, b = outs[0][0], outs[1][0]
    # the sweep schedule is the same red-black order whatever the blocking, so the
    # results agree to rounding (bitwise unless FMA contraction differs per variant)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(a).max()
