"""GPU parity of the online patch-dictionary update (Section IV-B: Eqs.
ADMM0 / sold_patch, ADMM1, subh) against the FP64 oracle. The code update
runs on BF16 MFMA as in the fixed-dictionary path; the dictionary step uses
split-BF16 MFMA products (FP32 accumulation), FP32 Cholesky factors and FP32
triangular solves. x must meet the BF16 path's 2e-3 relative l2, and so
must the learned dictionary G in relative Frobenius norm; the dictionary
step alone, on the same BF16 codes, must match FP64 to 1e-4 (the step's own
arithmetic on a well-conditioned system)."""
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


def _problem(N, K, S, A, cfg=3):
    x, psf, noise = synth.problem("smooth_disk", N, K, S, seed_config=cfg)
    y = model.measure(x, psf, noise, 30.0).astype(np.float32).astype(np.float64)
    D = synth.random_unit_atoms(synth.rng_for(cfg, 4), 64 * S, A)
    D = D / np.linalg.norm(D)                     # ||D||_F = 1 (Eq. patch_based_dic)
    D = D.astype(np.float32).astype(np.float64)
    return x, psf, y, D


# rho, lambda, beta for dictionaries of unit Frobenius norm: the soft
# threshold lambda / rho = 0.5
RHO, LAM, BETA = 1e-4, 5e-5, 500.0


def _sigma(N):
    """sigma proportional to the patch count J: with these images the codes
    reach ~100, the largest eigenvalue of Z Z^T grows like 1e4 J, and
    sigma = 1000 J keeps the condition number of Z Z^T + sigma I near 3-30
    (sigma = 1, the paper's setting for its data, gives ~1e6 here, beyond
    what FP32 products can resolve)."""
    return 1000.0 * (N // 4) ** 2


@pytest.mark.parametrize("N,K,S,A,iters,gtol", [
    (128, 3, 3, 128, 8, 2e-3),
    (64, 3, 4, 128, 6, 2e-3),
    (128, 3, 3, 256, 6, 2e-3),
    (64, 3, 4, 256, 5, 2e-3),
    (64, 2, 2, 64, 10, 2e-3),
    (128, 2, 2, 64, 10, 2e-3),
])
def test_patch_dictionary_learning_matches_oracle(N, K, S, A, iters, gtol):
    """x meets the BF16 bar (2e-3); the learned G (after the iters - 1
    dictionary steps the solve takes: the oracle's G of the next-to-last
    iteration) agrees within gtol, the BF16 code error carried through the
    dictionary steps (the D-step on identical codes agrees to 3-7e-7, next
    test)."""
    sigma = _sigma(N)
    print(f"patch dictionary learning N={N} K={K} S={S} A={A} iters={iters} sigma={sigma}",
          flush=True)
    x, psf, y, D = _problem(N, K, S, A)
    alg = admm.PatchADMM(psf, D, 8, 4, LAM, RHO, BETA, tier="freq", dict_update=True,
                         sigma=sigma)
    gs = []
    ref = alg.run(y, iters, callback=lambda it, *a: gs.append(alg.g.copy()))[0]
    g_ref = gs[iters - 2]
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=sigma)
    got = _np(plan.solve(_t(y), iters))
    g = _np(plan.dictionary())
    ex = admm.rel_l2(got, ref)
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    moved = np.linalg.norm(g_ref - D)
    print(f"  x rel_l2 {ex:.3e}  G rel {eg:.3e} (G moved {moved:.3e} from D; ||G||_F gpu "
          f"{np.linalg.norm(g):.6f})", flush=True)
    assert moved > 1e-3                 # the dictionary does change
    assert abs(np.linalg.norm(g) - 1.0) < 1e-5
    parity.check(got, ref, 2e-3, label="x")
    parity.check(g, g_ref, gtol, label="G")


def test_patch_dictionary_learning_full_size_1024():
    """The paper's patch configuration: 1024^2 x 3 planes, 8 x 8 x 3 patches
    at stride 4 (J = 65536), 256 atoms; 3 iterations (two dictionary
    steps)."""
    N, K, S, A, iters = 1024, 3, 3, 256, 3
    sigma = _sigma(N)
    print(f"patch dictionary learning N={N} A={A} iters={iters}", flush=True)
    x, psf, y, D = _problem(N, K, S, A)
    alg = admm.PatchADMM(psf, D, 8, 4, LAM, RHO, BETA, tier="freq", dict_update=True,
                         sigma=sigma)
    gs = []
    ref = alg.run(y, iters, callback=lambda it, *a: gs.append(alg.g.copy()))[0]
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=sigma)
    got = _np(plan.solve(_t(y), iters))
    g = _np(plan.dictionary())
    ex = admm.rel_l2(got, ref)
    eg = np.linalg.norm(g - gs[iters - 2]) / np.linalg.norm(gs[iters - 2])
    print(f"  x rel_l2 {ex:.3e}  G rel {eg:.3e}", flush=True)
    parity.check(got, ref, 2e-3, label="x")
    parity.check(g, gs[iters - 2], 2e-3, label="G")


def _bf16(a):
    """Round to the nearest BF16 value, ties to even (the code update's
    operand rounding)."""
    u = np.asarray(a, dtype=np.float32).view(np.uint32).astype(np.uint64)
    u = (u + 0x7FFF + ((u >> 16) & 1)) >> 16 << 16
    return u.astype(np.uint32).view(np.float32).astype(np.float64)


@pytest.mark.parametrize("N,K,S,A,sigma_kind,tol", [
    (64, 2, 2, 64, "scaled", 1e-4), (64, 3, 3, 256, "scaled", 1e-4),
    (128, 3, 4, 128, "scaled", 1e-4),
    (64, 2, 2, 64, "paper", 2e-3), (64, 3, 3, 256, "paper", 2e-3), (128, 4, 4, 128, "paper", 2e-3)])
def test_patch_dictionary_first_step_on_bf16_codes(N, K, S, A, sigma_kind, tol):
    """The first dictionary step, isolated from the BF16 code error: with
    two iterations the GPU takes one D, G, E step on z^1 = M1 e (w = 0,
    e = P x^1), whose operands M1 and e are BF16. The same step in FP64 on
    codes formed from BF16-rounded M1 and e (x^1 from the FP64 oracle) must
    give the GPU's G: the GPU's step runs in FP64 on its FP32 x and codes,
    which differ from the oracle's by FP32 rounding and the FP32
    accumulation of the code products. With sigma = 1000 J the step matches
    to 1e-4. At the paper's sigma = 1, Z Z^T + sigma I has condition numbers
    1e5 .. 6e6 here, and the FP32-level difference of x^1 (4e-7) flips the
    BF16 rounding of a few patch samples: perturbing the oracle's own x^1 by
    4e-7 moves its G by 3e-6 .. 1e-3 in these cases, so the bar is the BF16
    path's 2e-3."""
    sigma = _sigma(N) if sigma_kind == "scaled" else 1.0
    x, psf, y, D = _problem(N, K, S, A)
    alg = admm.PatchADMM(psf, D, 8, 4, LAM, RHO, BETA, tier="freq", dict_update=True,
                         sigma=sigma)
    x1 = alg.x_update(alg.solver.data_term(y), np.zeros((A, alg.P.J)))
    n = 64 * S
    M1 = np.linalg.solve(RHO * np.eye(n) + D @ D.T, D).T          # D^T (rho I + D D^T)^-1
    z1 = _bf16(M1) @ _bf16(alg.P.extract(x1))
    d = alg.d_update(x1, z1)
    g_ref = alg.g_update(d)
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=sigma)
    plan.solve(_t(y), 2)
    g = _np(plan.dictionary())
    eg = np.linalg.norm(g - g_ref) / np.linalg.norm(g_ref)
    moved = np.linalg.norm(g_ref - D)
    print(f"first step N={N} S={S} A={A} sigma={sigma:g}: G rel {eg:.3e} (step {moved:.3e})",
          flush=True)
    parity.check(g, g_ref, tol, label="G")


@pytest.mark.parametrize("N,K,S,A", [(64, 3, 3, 128), (128, 3, 3, 256)])
def test_patch_dictionary_learning_at_sigma_1(N, K, S, A):
    """The paper's sigma = 1 (the library default), 3 iterations (two
    dictionary steps of the FP64 D-step): x within the BF16 bar. Each step
    moves G by 0.04 .. 0.9 at this sigma and amplifies the BF16 code error
    (the learned G differs from the oracle's by 1e-2 .. 3e-2 after two steps,
    x by 3e-4), so x is the compared result."""
    x, psf, y, D = _problem(N, K, S, A)
    alg = admm.PatchADMM(psf, D, 8, 4, LAM, RHO, BETA, tier="freq", dict_update=True,
                         sigma=1.0)
    ref = alg.run(y, 3)[0]
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True)
    got = _np(plan.solve(_t(y), 3))
    print(f"sigma = 1, N={N} S={S} A={A}: psnr gpu {admm.psnr(got, x):.2f} dB, oracle "
          f"{admm.psnr(ref, x):.2f} dB", flush=True)
    parity.check(got, ref, 2e-3, label="x")


def test_patch_dictionary_huge_sigma_is_the_fixed_dictionary_run():
    """sigma -> infinity keeps G = D (||D||_F = 1): the learning plan then
    reproduces the fixed-dictionary plan (its code tables are rebuilt on the
    GPU in FP32 instead of on the host in FP64, hence the BF16 tolerance)."""
    x, psf, y, D = _problem(64, 3, 3, 128)
    fixed = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D))
    learn = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                     sigma=1e12)
    a = _np(fixed.solve(_t(y), 8))
    b = _np(learn.solve(_t(y), 8))
    err = admm.rel_l2(b, a)
    dg = np.abs(_np(learn.dictionary()) - D).max()
    print(f"huge sigma: rel_l2 vs fixed {err:.3e}, max |G - D| {dg:.3e}", flush=True)
    parity.check(b, a, 2e-3)
    assert dg < 1e-6


def test_patch_dictionary_solves_restart_from_the_plan_dictionary():
    """Every solve starts from the plan's dictionary: two solves agree
    bitwise (no atomics anywhere on the path), also after a shorter solve."""
    x, psf, y, D = _problem(64, 2, 2, 64)
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=_sigma(64))
    yt = _t(y)
    a = plan.solve(yt, 6).clone()
    ga = plan.dictionary().clone()
    plan.solve(yt, 3)
    b = plan.solve(yt, 6)
    gb = plan.dictionary()
    torch.cuda.synchronize()
    assert torch.equal(a, b)
    assert torch.equal(ga, gb)


@pytest.mark.skip(reason="capturing a learning patch plan into a graph ended in a host "
                  "segmentation fault inside batch creation, in a variant that rebuilt M1 on a "
                  "side stream (since taken out); the cause was not found, and graph capture of "
                  "dictionary-learning plans is refused (next test)")
def test_patch_dictionary_learning_in_a_captured_batch():
    """A captured and replayed batch of a learning plan (eager work between
    the replays) equals the lone solve bit for bit."""
    x, psf, y, D = _problem(64, 2, 2, 64)
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=_sigma(64))
    yt = _t(y)
    ref = plan.solve(yt, 6).clone()
    torch.cuda.synchronize()
    xs = torch.full_like(ref, float("nan"))
    b = cip.Batch([(plan, yt, 6, xs)], n_streams=1, graph=True)
    for rep in range(3):
        xs.fill_(float("nan"))
        b.launch()
        torch.cuda.synchronize()
        assert torch.equal(xs, ref), rep


def test_dictionary_learning_plans_are_not_captured():
    """Graph capture of dictionary-learning plans is refused before any
    capture starts (CIP_EUNSUPPORTED); a direct batch still runs them and
    equals the lone solve."""
    x, psf, y, D = _problem(64, 2, 2, 64)
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=_sigma(64))
    yt = _t(y)
    ref = plan.solve(yt, 6).clone()
    torch.cuda.synchronize()
    xs = torch.full_like(ref, float("nan"))
    with pytest.raises(cip.CipError) as e:
        cip.Batch([(plan, yt, 6, xs)], n_streams=1, graph=True)
    assert e.value.code == -2
    b = cip.Batch([(plan, yt, 6, xs)], n_streams=1, graph=False)
    b.launch()
    torch.cuda.synchronize()
    assert torch.equal(xs, ref)


def test_patch_dictionary_learning_1024_100_iterations_stays_feasible():
    """The timed learning configuration (1024^2 x 3, A = 256, the paper's
    sigma = 1, 100 iterations), beyond what the oracle runs in seconds:
    properties that hold at any size. G has unit Frobenius norm (Eq.
    patch_based_dic), x is finite, and the dictionary moved."""
    x, psf, y, D = _problem(1024, 3, 3, 256)
    plan = cip.Plan(_t(psf), "patch", RHO, LAM, BETA, dictionary=_t(D), dict_update=True,
                    sigma=1.0)
    got = _np(plan.solve(_t(y), 100))
    g = _np(plan.dictionary())
    moved = np.linalg.norm(g - D)
    print(f"patch 1024^2 learning x 100: ||G||_F {np.linalg.norm(g):.7f}, G moved {moved:.3e}",
          flush=True)
    assert np.isfinite(got).all()
    assert abs(np.linalg.norm(g) - 1.0) < 1e-5
    assert moved > 1e-3
