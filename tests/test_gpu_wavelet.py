"""GPU parity of the wavelet (x) DCT analysis prior (Section V-A's
Kronecker basis: 2D Symmlet-8 wavelet per plane, orthonormal DCT along the
bands; Algorithm 1 with Phi = l1) against the FP64 oracle, to the FP32
tolerance 1e-4 (relative l2 of x)."""
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


def _problem(N1, N2, K, S, cfg=10):
    x, psf, noise = synth.problem("smooth_disk", max(N1, N2), K, S, seed_config=cfg)
    if (N1, N2) != x.shape[1:]:
        x, psf = x[:, :N1, :N2].copy(), psf[:, :, :N1, :N2].copy()
        psf /= psf.sum(axis=(2, 3), keepdims=True)
        noise = noise[:, :N1, :N2]
    hx = model.forward(x, psf)
    y = hx + model.snr_noise_scale(hx, 30.0)[:, None, None] * noise
    return x, psf, y.astype(np.float32).astype(np.float64)


@pytest.mark.parametrize("N1,N2,K,S,levels,iters", [
    (64, 64, 3, 3, 3, 20), (128, 64, 2, 2, 4, 15), (32, 32, 1, 1, 2, 25),
    (384, 384, 3, 3, 3, 8), (256, 256, 3, 5, 5, 10), (16, 16, 2, 3, 1, 12),
    (64, 64, 3, 3, 6, 10), (256, 256, 3, 3, 3, 100),
])
def test_wavelet_dct_solve_matches_oracle(N1, N2, K, S, levels, iters):
    print(f"wdct3d N1={N1} N2={N2} K={K} S={S} levels={levels} iters={iters}", flush=True)
    x, psf, y = _problem(N1, N2, K, S)
    lam, rho, beta = 1e-2, 0.1, 1.0
    ref = admm.AnalysisADMM(psf, "wdct3d", lam, rho, beta, tier="freq", levels=levels).run(y, iters)[0]
    plan = cip.Plan(_t(psf), "wdct3d", rho, lam, beta, wt_levels=levels)
    got = _np(plan.solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB", flush=True)
    parity.check(got, ref, 1e-4)


def test_wavelet_dct_full_size_1024():
    """The precision workload's shape: 1024^2 x 3 planes, K = 3, 3 levels."""
    x, psf, y = _problem(1024, 1024, 3, 3)
    lam, rho, beta = 1e-2, 0.1, 1.0
    ref = admm.AnalysisADMM(psf, "wdct3d", lam, rho, beta, tier="freq").run(y, 4)[0]
    plan = cip.Plan(_t(psf), "wdct3d", rho, lam, beta)
    got = _np(plan.solve(_t(y), 4))
    err = admm.rel_l2(got, ref)
    print(f"wdct3d 1024^2 x 3, 4 iterations: rel_l2 {err:.3e}", flush=True)
    parity.check(got, ref, 1e-4)


def test_wavelet_dct_differs_from_dct3d_and_repeats_bitwise():
    """A different transform gives a different answer than the DCT3D prior,
    and two solves on one plan agree bitwise (the state restarts)."""
    x, psf, y = _problem(64, 64, 3, 3)
    plan = cip.Plan(_t(psf), "wdct3d", 0.1, 1e-2, 1.0)
    yt = _t(y)
    a = plan.solve(yt, 10).clone()
    b = plan.solve(yt, 10)
    d = cip.Plan(_t(psf), "dct3d", 0.1, 1e-2, 1.0).solve(yt, 10)
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert float(torch.linalg.vector_norm(a - d) / torch.linalg.vector_norm(d)) > 1e-3
