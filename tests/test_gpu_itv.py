"""GPU parity of the isotropic-TV prior (T = I, t-update = TV proximal map by
Chambolle's algorithm with a warm-started dual) against the FP64 oracle;
FP32 path, 1e-4 relative l2 on x after a fixed iteration count."""
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


def _problem(kind, N, K, S, cfg=12):
    x, psf, noise = synth.problem(kind, N, K, S, seed_config=cfg)
    hx = model.forward(x, psf)
    y = (hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise)
    return x, psf, y.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("kind,N,K,S,iters,inner", [("rects_gauss", 64, 2, 2, 20, 20),
                                                    ("smooth_disk", 64, 3, 3, 10, 20),
                                                    ("smooth_disk", 128, 3, 3, 8, 10),
                                                    ("smooth_disk", 128, 3, 3, 100, 20),
                                                    ("rects_gauss", 256, 2, 3, 5, 20),
                                                    ("smooth_disk", 384, 3, 3, 4, 15),
                                                    ("smooth_disk", 64, 3, 3, 1, 20),
                                                    ("rects_gauss", 16, 2, 2, 6, 3),
                                                    ("smooth_disk", 32, 2, 2, 5, 1),
                                                    ("rects_gauss", 64, 2, 2, 6, 7)])
def test_itv_solve_matches_oracle(kind, N, K, S, iters, inner):
    print(f"itv2d {kind} N={N} K={K} S={S} iters={iters} inner={inner}", flush=True)
    x, psf, y = _problem(kind, N, K, S)
    lam, rho = 1e-3, 1e-2
    ref = admm.AnalysisADMM(psf, "itv2d", lam, rho, 1.0, tier="freq", inner=inner).run(y, iters)[0]
    got = _np(cip.Plan(_t(psf), "itv2d", rho, lam, 1.0, tv_inner=inner).solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB oracle "
          f"{admm.psnr(ref, x):.2f} dB", flush=True)
    parity.check(got, ref, 1e-4)


def test_itv_differs_from_anisotropic():
    x, psf, y = _problem("rects_gauss", 64, 2, 2)
    lam, rho = 1e-2, 1e-2
    ref = admm.AnalysisADMM(psf, "itv2d", lam, rho, 1.0, tier="freq").run(y, 30)[0]
    gi = _np(cip.Plan(_t(psf), "itv2d", rho, lam, 1.0).solve(_t(y), 30))
    ga = _np(cip.Plan(_t(psf), "tv2d", rho, lam, 1.0).solve(_t(y), 30))
    parity.check(gi, ref, 1e-4)
    assert admm.rel_l2(ga, gi) > 1e-3


def test_itv_repeat_solve_and_odd_launch_count():
    """inner = 3 takes one Chambolle launch per ADMM iteration, so the dual
    changes buffer from one iteration to the next; a second solve on the same
    plan restarts from p = 0 and gives the same x."""
    x, psf, y = _problem("smooth_disk", 64, 2, 2)
    lam, rho = 1e-3, 1e-2
    ref = admm.AnalysisADMM(psf, "itv2d", lam, rho, 1.0, tier="freq", inner=3).run(y, 7)[0]
    plan = cip.Plan(_t(psf), "itv2d", rho, lam, 1.0, tv_inner=3)
    a = _np(plan.solve(_t(y), 7))
    b = _np(plan.solve(_t(y), 7))
    parity.check(a, ref, 1e-4)
    assert np.array_equal(a, b)


def test_itv_rejects_zero_lambda():
    psf = np.zeros((1, 1, 32, 32))
    psf[0, 0, 0, 0] = 1.0
    with pytest.raises(RuntimeError):
        cip.Plan(_t(psf), "itv2d", 1e-2, 0.0, 1.0)


# ---------------------------------------------------------------- TV coupled along the planes
@pytest.mark.parametrize("kind,N,K,S,iters,inner", [("rects_gauss", 64, 2, 2, 20, 20),
                                                    ("smooth_disk", 64, 3, 3, 10, 20),
                                                    ("smooth_disk", 128, 3, 3, 8, 10),
                                                    ("smooth_disk", 128, 3, 3, 100, 20),
                                                    ("rects_gauss", 16, 2, 2, 6, 3),
                                                    ("smooth_disk", 48 * 8, 3, 3, 4, 15),
                                                    ("rects_gauss", 64, 2, 1, 6, 7),
                                                    ("rects_gauss", 64, 4, 4, 6, 10),
                                                    ("smooth_disk", 32, 5, 5, 5, 6),
                                                    ("rects_gauss", 64, 8, 8, 6, 10),
                                                    ("smooth_disk", 256, 2, 6, 3, 20),
                                                    ("smooth_disk", 64, 3, 3, 1, 20),
                                                    ("smooth_disk", 1024, 3, 3, 2, 10)])
def test_itv3_solve_matches_oracle(kind, N, K, S, iters, inner):
    """Every plane count 1 .. 8 (32 x 32 tiles for S <= 3 where the grid
    allows, 16 x 16 otherwise), inner counts that split unevenly over the
    launches of 5, grids from 16^2 (halo wider than a third of the grid) to
    1024^2."""
    print(f"itv3d {kind} N={N} K={K} S={S} iters={iters} inner={inner}", flush=True)
    x, psf, y = _problem(kind, N, K, S)
    lam, rho = 1e-3, 1e-2
    ref = admm.AnalysisADMM(psf, "itv3d", lam, rho, 1.0, tier="freq", inner=inner).run(y, iters)[0]
    got = _np(cip.Plan(_t(psf), "itv3d", rho, lam, 1.0, tv_inner=inner).solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB oracle "
          f"{admm.psnr(ref, x):.2f} dB", flush=True)
    parity.check(got, ref, 1e-4)


def test_itv3_differs_from_per_plane_itv_and_repeats():
    """On planes that differ, the band-coupled prior gives another answer
    than the per-plane one; a second solve on the same plan restarts from
    p = 0 and gives the same x."""
    x, psf, y = _problem("rects_gauss", 64, 3, 3)
    lam, rho = 1e-2, 1e-2
    ref = admm.AnalysisADMM(psf, "itv3d", lam, rho, 1.0, tier="freq", inner=3).run(y, 9)[0]
    plan = cip.Plan(_t(psf), "itv3d", rho, lam, 1.0, tv_inner=3)
    a = _np(plan.solve(_t(y), 9))
    b = _np(plan.solve(_t(y), 9))
    g2 = _np(cip.Plan(_t(psf), "itv2d", rho, lam, 1.0, tv_inner=3).solve(_t(y), 9))
    parity.check(a, ref, 1e-4)
    assert np.array_equal(a, b)
    assert admm.rel_l2(g2, a) > 1e-3


def test_itv3_rejects_zero_lambda_and_bad_inner_count():
    psf = np.zeros((2, 2, 32, 32))
    psf[0, 0, 0, 0] = psf[1, 1, 0, 0] = 1.0
    with pytest.raises(RuntimeError):
        cip.Plan(_t(psf), "itv3d", 1e-2, 0.0, 1.0)
    with pytest.raises(RuntimeError):
        cip.Plan(_t(psf), "itv3d", 1e-2, 1e-3, 1.0, tv_inner=10001)


@pytest.mark.parametrize("prior,N1,N2,K,S,iters,inner", [("itv2d", 64, 128, 2, 2, 6, 7),
                                                         ("itv2d", 384, 256, 3, 3, 3, 10),
                                                         ("itv3d", 128, 64, 2, 3, 6, 7),
                                                         ("itv3d", 16, 64, 2, 2, 5, 6),
                                                         ("itv3d", 256, 384, 3, 3, 3, 10),
                                                         ("itv3d", 64, 32, 4, 5, 4, 5)])
def test_itv_rectangular_grids(prior, N1, N2, K, S, iters, inner):
    """Grids with N1 != N2 (tile counts differ along the two axes; 16-row
    grids take 16 x 16 tiles): smooth bands blurred by defocus disks, 30 dB."""
    print(f"{prior} N1={N1} N2={N2} K={K} S={S} iters={iters} inner={inner}", flush=True)
    x = synth.smooth_images(synth.rng_for(12, 0), S, N1, N2).astype(np.float32).astype(np.float64)
    psf = synth.disk_psfs(K, S, N1, N2).astype(np.float32).astype(np.float64)
    noise = synth.unit_noise(synth.rng_for(12, 2), K, N1, N2).astype(np.float32).astype(np.float64)
    hx = model.forward(x, psf)
    y = (hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise).astype(np.float32)
    y = y.astype(np.float64)
    lam, rho = 1e-3, 1e-2
    ref = admm.AnalysisADMM(psf, prior, lam, rho, 1.0, tier="freq", inner=inner).run(y, iters)[0]
    got = _np(cip.Plan(_t(psf), prior, rho, lam, 1.0, tv_inner=inner).solve(_t(y), iters))
    parity.check(got, ref, 1e-4)
