"""GPU parity of the TV3D analysis prior (anisotropic TV along both image
axes plus a forward difference along the plane axis, Section III-A's
multidimensional derivative operators) against the FP64 oracle; FP32 path,
tolerance 1e-4 relative l2 on x after a fixed iteration count."""
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


def _problem(kind, N, K, S, cfg):
    x, psf, noise = synth.problem(kind, N, K, S, seed_config=cfg)
    hx = model.forward(x, psf)
    y = (hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise)
    return x, psf, y.astype(np.float32).astype(np.float64)


# serving-workload reading: lambda = 1e-3, rho = 1e-2, beta = 1
@pytest.mark.parametrize("N,K,S,iters,kind", [(64, 3, 3, 30, "smooth_disk"),
                                              (128, 5, 5, 15, "smooth_disk"),
                                              (64, 2, 2, 20, "rects_gauss"),
                                              (32, 8, 8, 8, "smooth_disk"),
                                              (16, 2, 3, 6, "rects_gauss"),
                                              (256, 3, 8, 5, "smooth_disk"),
                                              (64, 3, 3, 1, "smooth_disk")])
def test_tv3d_solve_matches_oracle(N, K, S, iters, kind):
    print(f"tv3d solve N={N} K={K} S={S} iters={iters} {kind}", flush=True)
    x, psf, y = _problem(kind, N, K, S, 5)
    lam, rho, beta = 1e-3, 1e-2, 1.0
    ref = admm.AnalysisADMM(psf, "tv3d", lam, rho, beta, tier="freq").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "tv3d", rho, lam, beta)
    got = _np(plan.solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB oracle {admm.psnr(ref, x):.2f}",
          flush=True)
    parity.check(got, ref, 1e-4)


def test_tv3d_single_plane_equals_tv2d():
    """With S = 1 there is no band difference: TV3D must reproduce TV2D (same
    Gram, same row arithmetic; the two kernels are compiled separately, so
    contraction into fused multiply-adds may differ in the last bit)."""
    x, psf, y = _problem("smooth_disk", 128, 3, 1, 6)
    a = cip.Plan(_t(psf), "tv3d", 1e-2, 1e-3, 1.0)
    b = cip.Plan(_t(psf), "tv2d", 1e-2, 1e-3, 1.0)
    ga = _np(a.solve(_t(y), 10))
    gb = _np(b.solve(_t(y), 10))
    parity.check(ga, gb, 1e-6)


def test_tv3d_band_coupling_matters():
    """The band term changes the answer for S > 1 (guards against the band
    update being skipped): TV3D and TV2D differ by far more than the FP32
    tolerance, and TV3D is the one that matches the oracle."""
    x, psf, y = _problem("smooth_disk", 64, 3, 3, 7)
    lam, rho = 1e-2, 1e-2
    ref3 = admm.AnalysisADMM(psf, "tv3d", lam, rho, 1.0, tier="freq").run(y, 20)[0]
    g3 = _np(cip.Plan(_t(psf), "tv3d", rho, lam, 1.0).solve(_t(y), 20))
    g2 = _np(cip.Plan(_t(psf), "tv2d", rho, lam, 1.0).solve(_t(y), 20))
    parity.check(g3, ref3, 1e-4)
    assert admm.rel_l2(g2, ref3) > 1e-3


@pytest.mark.parametrize("N,K,S,iters", [(1024, 3, 3, 3), (512, 8, 8, 2), (2048, 3, 3, 2)])
def test_tv3d_full_size(N, K, S, iters):
    """Serving-workload sizes (1024^2 and 2048^2 with K = S = 3, 512^2 with
    K = S = 8), a few iterations."""
    print(f"tv3d full size N={N} K={K} S={S} iters={iters}", flush=True)
    x, psf, y = _problem("smooth_disk", N, K, S, 5)
    ref = admm.AnalysisADMM(psf, "tv3d", 1e-3, 1e-2, 1.0, tier="freq").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "tv3d", 1e-2, 1e-3, 1.0)
    got = _np(plan.solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}", flush=True)
    parity.check(got, ref, 1e-4)
