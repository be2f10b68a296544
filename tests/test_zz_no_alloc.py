"""cip_solve_static (the entry point that allocates no device memory) against
cip_plan_create + cip_solve on caller memory: two calls in a row, the second
on a smaller problem, each equal to the plan-based solve (the same kernels on
the same data: bitwise) and within the FP32 parity bar."""
import numpy as np
import pytest
import torch

from tests import parity
from oracle import model
from paper_2006_08303_amd import cip, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _case(N, K, S, kind, cfg):
    x, psf, noise = synth.problem(kind, N, K, S, seed_config=cfg)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    return _t(psf), _t(y)


@pytest.mark.timeout(300)
def test_solve_static_equals_plan_solve_twice_shrinking():
    cases = [(512, 3, 3, "smooth_disk", 2, "dct2d", 0.1, 1e-2, 30),
             (128, 2, 3, "rects_gauss", 1, "tv2d", 1e-2, 1e-3, 20),
             (64, 3, 3, "smooth_disk", 4, "tv3d", 1e-2, 1e-3, 15)]
    for N, K, S, kind, cfg, prior, rho, lam, iters in cases:
        print(f"solve_static {prior} N={N} K={K} S={S} iters={iters}", flush=True)
        psf, y = _case(N, K, S, kind, cfg)
        got = cip.solve_static(psf, y, iters, prior, rho, lam, 1.0)
        ref = cip.Plan(psf, prior, rho, lam, 1.0).solve(y, iters)
        torch.cuda.synchronize()
        g, r = got.cpu().double().numpy(), ref.cpu().double().numpy()
        parity.check(g, r, 1e-4, label=f"static vs plan {prior} {N}")
        assert np.array_equal(g, r)
