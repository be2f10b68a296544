"""GPU parity of the patch-dictionary synthesis prior (Algorithm 2 with
Eq. solz_patch2) against the FP64 oracle. The sparse-code update runs on
BF16 MFMA with FP32 accumulation: x after the fixed iteration count must be
within 2e-3 relative l2 of the oracle (the tolerance stated for the BF16
dictionary path)."""
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


def _patch_problem(N, K, S, A, cfg=3):
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=cfg)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    D = synth.random_unit_atoms(synth.rng_for(cfg, 4), 64 * S, A)
    D = D.astype(np.float32).astype(np.float64)
    return x, psf, y, D


# config-3 reading: rho = 1e-4, lambda = 5e-6 (threshold lambda / rho = 0.05),
# beta = 500, c_P = 4
# Dictionaries are over- or under-complete (A != 64 S), so that rho I + D D^T
# is well conditioned; a random square dictionary makes it nearly singular
# (smallest eigenvalue ~1e-7) and BF16 operand rounding is then amplified.
@pytest.mark.parametrize("N,K,S,A,iters", [(64, 3, 3, 256, 20), (128, 3, 3, 256, 10),
                                           (256, 3, 3, 256, 5), (64, 2, 1, 128, 15),
                                           (64, 2, 2, 256, 15), (32, 3, 4, 128, 8),
                                           (64, 3, 3, 64, 10)])
def test_patch_solve_matches_oracle(N, K, S, A, iters):
    print(f"patch solve N={N} K={K} S={S} A={A} iters={iters}", flush=True)
    x, psf, y, D = _patch_problem(N, K, S, A)
    lam, rho, beta = 5e-6, 1e-4, 500.0
    ref = admm.PatchADMM(psf, D, 8, 4, lam, rho, beta, tier="freq").run(y, iters)[0]
    plan = cip.Plan(_t(psf), "patch", rho, lam, beta, dictionary=_t(D))
    got = _np(plan.solve(_t(y), iters))
    err = admm.rel_l2(got, ref)
    print(f"  rel_l2 = {err:.3e}  psnr gpu {admm.psnr(got, x):.2f} dB oracle "
          f"{admm.psnr(ref, x):.2f} dB", flush=True)
    parity.check(got, ref, 2e-3)


def test_patch_first_iterate_is_fp32_exact():
    """With one iteration the patch update has not run yet: x^1 is the
    x-update from z = 0 and must meet the FP32 tolerance."""
    x, psf, y, D = _patch_problem(64, 3, 3, 256)
    ref = admm.PatchADMM(psf, D, 8, 4, 5e-6, 1e-4, 500.0, tier="freq").run(y, 1)[0]
    plan = cip.Plan(_t(psf), "patch", 1e-4, 5e-6, 500.0, dictionary=_t(D))
    parity.check(_np(plan.solve(_t(y), 1)), ref, 1e-4)


def test_patch_full_size_1024():
    """Configuration of the precision workload: K = S = 3, 1024 x 1024,
    8 x 8 x 3 patches at stride 4 (J = 65536), 256 atoms; 4 iterations."""
    x, psf, y, D = _patch_problem(1024, 3, 3, 256)
    ref = admm.PatchADMM(psf, D, 8, 4, 5e-6, 1e-4, 500.0, tier="freq").run(y, 4)[0]
    plan = cip.Plan(_t(psf), "patch", 1e-4, 5e-6, 500.0, dictionary=_t(D))
    got = _np(plan.solve(_t(y), 4))
    err = admm.rel_l2(got, ref)
    print(f"1024^2 patch 4 iters: rel_l2 = {err:.3e}", flush=True)
    parity.check(got, ref, 2e-3)
