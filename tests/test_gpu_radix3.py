"""GPU parity on grids of 3 * 2^k points (384, 768, 1536), which the batch and
serving workloads draw: the transforms there start with a radix-12 stage in
registers (radix 3 inside) and continue with radices 4 and 2. FP32 paths
against the FP64 oracle: 1e-5 for single operator applications, 1e-4 on x
after a fixed iteration count."""
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


@pytest.mark.parametrize("K,S,N1,N2", [(2, 3, 384, 384), (3, 2, 768, 768), (2, 2, 1536, 1536),
                                       (2, 3, 384, 512), (3, 3, 256, 768), (1, 1, 1536, 2048)])
def test_forward_adjoint_radix3(K, S, N1, N2):
    print(f"forward/adjoint K={K} S={S} {N1}x{N2}", flush=True)
    rng = np.random.default_rng(21)
    psf = synth.gaussian_psfs(rng, K, S, N1, N2, sigma_range=(0.8, 3.0))
    psf = psf.astype(np.float32).astype(np.float64)
    x = rng.uniform(0, 1, (S, N1, N2)).astype(np.float32).astype(np.float64)
    y = rng.standard_normal((K, N1, N2)).astype(np.float32).astype(np.float64)
    plan = cip.Plan(_t(psf), "dct2d", 0.1, 0.01, 1.0)
    parity.check(_np(plan.forward(_t(x))), model.forward(x, psf), 1e-5)
    parity.check(_np(plan.adjoint(_t(y))), model.adjoint(y, psf), 1e-5)


def _problem(kind, N, K, S, cfg):
    x, psf, noise = synth.problem(kind, N, K, S, seed_config=cfg)
    hx = model.forward(x, psf)
    y = (hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise)
    return x, psf, y.astype(np.float32).astype(np.float64)


PARAMS = {"dct2d": (1e-2, 0.1), "tv2d": (1e-3, 1e-2), "tv3d": (1e-3, 1e-2)}


@pytest.mark.parametrize("prior,N,K,S,iters", [("dct2d", 384, 3, 3, 15), ("tv2d", 384, 2, 4, 12),
                                               ("tv3d", 384, 5, 5, 8), ("dct2d", 768, 3, 3, 5),
                                               ("tv3d", 768, 3, 3, 4), ("tv2d", 1536, 3, 3, 2)])
def test_solve_radix3(prior, N, K, S, iters):
    print(f"{prior} solve N={N} K={K} S={S} iters={iters}", flush=True)
    x, psf, y = _problem("smooth_disk", N, K, S, 8)
    lam, rho = PARAMS[prior]
    ref = admm.AnalysisADMM(psf, prior, lam, rho, 1.0, tier="freq").run(y, iters)[0]
    got = _np(cip.Plan(_t(psf), prior, rho, lam, 1.0).solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}", flush=True)
    parity.check(got, ref, 1e-4)


def test_rectangular_radix3_tv():
    """N1 = 384, N2 = 768 (non-square, both with a factor 3), TV2D."""
    rng = np.random.default_rng(22)
    K, S, N1, N2 = 2, 3, 384, 768
    psf = synth.gaussian_psfs(rng, K, S, N1, N2, sigma_range=(0.8, 2.5))
    psf = psf.astype(np.float32).astype(np.float64)
    x = rng.uniform(0, 1, (S, N1, N2))
    y = (model.forward(x, psf) + 0.01 * rng.standard_normal((K, N1, N2)))
    y = y.astype(np.float32).astype(np.float64)
    ref = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="freq").run(y, 10)[0]
    got = _np(cip.Plan(_t(psf), "tv2d", 1e-2, 1e-3, 1.0).solve(_t(y), 10))
    parity.check(got, ref, 1e-4)


def test_conv_radix3():
    """Convolutional-dictionary prior on 384 x 384."""
    x, psf, noise = synth.problem("smooth_disk", 384, 3, 3, seed_config=8)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    filt = synth.random_unit_filters(synth.rng_for(8, 5), 8, 5).astype(np.float32).astype(np.float64)
    lam, rho, beta = 1.875e-6, 1e-4, 8.0
    ref = admm.ConvADMM(psf, filt, lam, rho, beta, tier="freq").run(y, 4)[0]
    got = _np(cip.Plan(_t(psf), "conv2d", rho, lam, beta, filters=_t(filt)).solve(_t(y), 4))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}", flush=True)
    parity.check(got, ref, 1e-4)


def test_patch_rejects_radix3():
    x, psf, _ = synth.problem("smooth_disk", 384, 3, 3, seed_config=8)
    D = synth.random_unit_atoms(synth.rng_for(8, 4), 192, 256)
    with pytest.raises(cip.CipError) as e:
        cip.Plan(_t(psf), "patch", 1e-4, 5e-6, 500.0, dictionary=_t(D))
    assert e.value.code == -2
