"""GPU parity of the 3D DCT analysis prior (2D DCT of every plane followed by
the DCT along the band axis) against the FP64 oracle; FP32 path, 1e-4
relative l2 on x after a fixed iteration count."""
import numpy as np
import pytest
import torch

from tests import parity
from oracle import admm, model
from paper_2006_08303_amd import cip, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _problem(N, K, S, cfg=11):
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=cfg)
    hx = model.forward(x, psf)
    y = (hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise)
    return x, psf, y.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("N,K,S,iters", [(64, 3, 3, 30), (128, 5, 5, 12), (64, 2, 1, 10),
                                         (256, 3, 8, 6), (384, 3, 3, 5), (1024, 3, 3, 3),
                                         (32, 8, 8, 10), (64, 3, 3, 1), (256, 3, 3, 100)])
def test_dct3d_solve_matches_oracle(N, K, S, iters):
    print(f"dct3d N={N} K={K} S={S} iters={iters}", flush=True)
    x, psf, y = _problem(N, K, S)
    lam, rho = 1e-2, 0.1
    ref = admm.AnalysisADMM(psf, "dct3d", lam, rho, 1.0, tier="freq").run(y, iters)[0]
    got = _np(cip.Plan(_t(psf), "dct3d", rho, lam, 1.0).solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB oracle "
          f"{admm.psnr(ref, x):.2f} dB", flush=True)
    parity.check(got, ref, 1e-4)


def test_dct3d_single_plane_equals_dct2d():
    """With S = 1 the band DCT is the identity: DCT3D reproduces DCT2D."""
    x, psf, y = _problem(128, 3, 1)
    a = _np(cip.Plan(_t(psf), "dct3d", 0.1, 1e-2, 1.0).solve(_t(y), 10))
    b = _np(cip.Plan(_t(psf), "dct2d", 0.1, 1e-2, 1.0).solve(_t(y), 10))
    parity.check(a, b, 1e-6)


def test_dct3d_adaptive_matches_oracle():
    x, psf, y = _problem(128, 3, 3)
    ref, rinfo = admm.AnalysisADMM(psf, "dct3d", 1e-2, 10.0, 1.0, tier="freq").run_adaptive(
        y, 200, every=5, tol=1e-3)
    plan = cip.Plan(_t(psf), "dct3d", 10.0, 1e-2, 1.0, adaptive=True)
    got, ginfo = plan.solve_adaptive(_t(y), 200, every=5, tol=1e-3)
    print(f"oracle {rinfo['iters']} {rinfo['rho']}; gpu {ginfo['iters']} {ginfo['rho']}", flush=True)
    assert ginfo["iters"] == rinfo["iters"] and ginfo["rho"] == pytest.approx(rinfo["rho"])
    parity.check(_np(got), ref, 1e-4)
