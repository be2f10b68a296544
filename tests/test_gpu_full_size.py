"""GPU parity at the configured iteration counts and full sizes.

* Headline shape (K = S = 3, 1024 x 1024, defocus disks, 30 dB): DCT-l1 and
  anisotropic TV after 100 iterations (Algorithm 1), in every row-pass shape
  the autotuner can pick (so whichever shape the benchmark times is covered),
  against the FP64 oracle run in the test.
* Precision workload (Algorithm 2, rho = 1e-4): the patch dictionary
  (8 x 8 x 3 patches, stride 4, 256 atoms, BF16 MFMA code update) and the
  common convolutional dictionary (32 filters of 11 x 11) after 100
  iterations, at 256^2 / 128^2 against the oracle run in the test and at
  1024^2 against the stored oracle sample in tests/golden (written by
  tests/golden/make_precision_1024.py, which calls only the oracle).
* Small case (K = S = 2, 64 x 64, rectangles, Gaussian kernels, TV,
  50 iterations) against the oracle's dense tier: the x-update by Cholesky
  of the assembled normal matrix (Eq. solx_Trans) instead of the
  per-frequency tier.

Bounds (tests/parity.py): relative l2 below the path's tolerance (1e-4 FP32,
2e-3 BF16 dictionary) and max |got - ref| <= 10 tol max |ref|.
"""
import importlib.util
import os

import numpy as np
import pytest
import torch

from tests import parity
from oracle import admm, model
from paper_2006_08303_amd import cip, synth

pytestmark = pytest.mark.gpu
DEV = torch.device("cuda:0")
HERE = os.path.dirname(os.path.abspath(__file__))


def _t(a):
    return torch.tensor(np.ascontiguousarray(a), dtype=torch.float32, device=DEV)


def _np(t):
    torch.cuda.synchronize()
    return t.cpu().double().numpy()


def _headline(N=1024, K=3, S=3):
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=3)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    return x, psf, y


# row pairs per work-group x points per thread: every shape the autotuner times
ROW_SHAPES = [(4, 16), (4, 8), (2, 16), (2, 8)]


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prior,lam,rho", [("dct2d", 1e-2, 0.1), ("tv2d", 1e-3, 1e-2),
                                           ("tv3d", 1e-3, 1e-2)])
def test_headline_1024_100_iterations(prior, lam, rho):
    N, K, S, iters = 1024, 3, 3, 100
    print(f"headline {prior} {N}^2 K=S={S}, {iters} iterations", flush=True)
    x, psf, y = _headline(N, K, S)
    ref = admm.AnalysisADMM(psf, prior, lam, rho, 1.0, tier="freq").run(y, iters)[0]
    print(f"  oracle psnr vs truth {admm.psnr(ref, x):.2f} dB", flush=True)
    plan = cip.Plan(_t(psf), prior, rho, lam, 1.0)
    yt = _t(y)
    first = None
    for np_, ppt in ROW_SHAPES:
        plan.set_tuning(np_, ppt)
        got = _np(plan.solve(yt, iters))
        parity.check(got, ref, 1e-4, label=f"{prior} row shape {np_}x{ppt}")
        if first is None:
            first = got
    # the shape changes only the order of the row transforms' arithmetic
    parity.check(first, ref, 1e-4, label=f"{prior} default shape")


@pytest.mark.timeout(600)
def test_patch_256_100_iterations():
    """Precision-workload parameters on a 256^2 grid, 100 iterations."""
    N, K, S, A, iters = 256, 3, 3, 256, 100
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=3)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    D = synth.random_unit_atoms(synth.rng_for(3, 4), 64 * S, A).astype(np.float32).astype(np.float64)
    ref = admm.PatchADMM(psf, D, 8, 4, 5e-6, 1e-4, 500.0, tier="freq").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "patch", 1e-4, 5e-6, 500.0, dictionary=_t(D))
    got = _np(plan.solve(_t(y), iters))
    print(f"  psnr vs truth: gpu {admm.psnr(got, x):.2f} dB, oracle {admm.psnr(ref, x):.2f} dB",
          flush=True)
    parity.check(got, ref, 2e-3, label="patch 256^2 x 100")


@pytest.mark.timeout(600)
def test_conv_128_100_iterations():
    """Precision-workload parameters (32 filters of 11 x 11) on a 128^2 grid,
    100 iterations."""
    N, K, S, M, L, iters = 128, 3, 3, 32, 11, 100
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=3)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    filt = synth.random_unit_filters(synth.rng_for(3, 5), M, L).astype(np.float32).astype(np.float64)
    ref = admm.ConvADMM(psf, filt, 1.875e-6, 1e-4, 8.0, tier="freq").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "conv2d", 1e-4, 1.875e-6, 8.0, filters=_t(filt))
    got = _np(plan.solve(_t(y), iters))
    print(f"  psnr vs truth: gpu {admm.psnr(got, x):.2f} dB, oracle {admm.psnr(ref, x):.2f} dB",
          flush=True)
    parity.check(got, ref, 1e-4, label="conv 128^2 x 100")


def _golden_module():
    spec = importlib.util.spec_from_file_location(
        "make_precision_1024", os.path.join(HERE, "golden", "make_precision_1024.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


@pytest.mark.timeout(600)
@pytest.mark.parametrize("which,tol", [("patch", 2e-3), ("conv", 1e-4)])
def test_precision_workload_1024_100_iterations(which, tol):
    """K = S = 3, 1024 x 1024, 100 iterations against the stored oracle
    sample (whole rows and columns including the borders, random pixels)."""
    gm = _golden_module()
    gold = np.load(os.path.join(HERE, "golden", f"precision_1024_{which}.npz"))
    x, psf, y, dic = gm.inputs(which)
    # the inputs must be the ones the stored x was computed from
    assert np.isclose(y.sum(), float(gold["y_sum"]), rtol=1e-12, atol=0.0)
    assert np.isclose((y * y).sum(), float(gold["y_sumsq"]), rtol=1e-12, atol=0.0)
    assert np.isclose(dic.sum(), float(gold["dic_sum"]), rtol=1e-12, atol=1e-12)
    p = gm.PARAMS[which]
    iters = int(gold["iters"])
    if which == "patch":
        plan = cip.Plan(_t(psf), "patch", p["rho"], p["lam"], p["beta"], dictionary=_t(dic))
    else:
        plan = cip.Plan(_t(psf), "conv2d", p["rho"], p["lam"], p["beta"], filters=_t(dic))
    got = _np(plan.solve(_t(y), iters))
    rows, cols, pix = gold["rows"], gold["cols"], gold["pix"]
    g = np.concatenate([got[:, rows, :].ravel(), got[:, :, cols].ravel(),
                        got.reshape(got.shape[0], -1)[:, pix].ravel()])
    r = np.concatenate([gold["x_rows"].ravel(), gold["x_cols"].ravel(),
                        gold["x_pix"].ravel()]).astype(np.float64)
    print(f"  {which}: psnr vs truth gpu {admm.psnr(got, x):.2f} dB, oracle "
          f"{float(gold['psnr_truth']):.2f} dB", flush=True)
    parity.check(g, r, tol, label=f"{which} 1024^2 x {iters} (sample)")
    # whole-image properties: the norm and the plane means
    nrm = float(gold["norm"])
    assert abs(np.linalg.norm(got) - nrm) <= tol * nrm
    assert np.max(np.abs(got.mean(axis=(1, 2)) - gold["plane_mean"])) <= \
        parity.C_ELEMENT * tol * float(gold["maxabs"])


@pytest.mark.timeout(600)
def test_small_case_against_dense_tier():
    """K = S = 2, 64 x 64 rectangles with Gaussian kernels, TV (lambda = 1e-3,
    rho = 1e-2), 50 iterations; the oracle's x-update is the dense tier
    (assembled normal matrix, Cholesky, null-space projector for the
    singular DC block)."""
    N, K, S, iters = 64, 2, 2, 50
    x, psf, noise = synth.problem("rects_gauss", N, K, S, seed_config=1)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    ref = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="dense").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "tv2d", 1e-2, 1e-3, 1.0)
    got = _np(plan.solve(_t(y), iters))
    print(f"  psnr vs truth: gpu {admm.psnr(got, x):.2f} dB, oracle {admm.psnr(ref, x):.2f} dB",
          flush=True)
    parity.check(got, ref, 1e-4, label="tv2d 64^2 x 50 vs dense tier")
