"""Pins of the FP64 oracle against facts fixed by mathematics or by
independent libraries (not against the oracle itself).

Each test names the paper passage whose oracle function it pins."""
import math

import numpy as np
import pytest
import scipy.fft
import scipy.ndimage
import scipy.optimize

from oracle import admm, model, priors, xupdate
from paper_2006_08303_amd import synth


def _rng(i=0):
    return np.random.default_rng(12345 + i)


def _dft_matrix(n):
    """Explicit DFT matrix from complex exponentials (no FFT library)."""
    k = np.arange(n)
    return np.exp(-2j * math.pi * np.outer(k, k) / n)


def _small_problem(K=2, S=2, N1=8, N2=8, seed=0, gauss=True):
    rng = _rng(seed)
    if gauss:
        psf = synth.gaussian_psfs(rng, K, S, N1, N2, sigma_range=(0.6, 1.5))
    else:
        psf = synth.disk_psfs(K, S, N1, N2, r_max=2.0)
    x = rng.uniform(0, 1, (S, N1, N2))
    return x, psf


# ------------------------------------------------------------------ forward model
def test_conv_matches_scipy_wrap():
    """Eq. forward model: circular convolution equals scipy.ndimage's
    wrap-mode convolution with the kernel re-centred."""
    rng = _rng(1)
    N1, N2 = 12, 10
    x = rng.standard_normal((N1, N2))
    h = np.zeros((N1, N2))
    taps = {(0, 0): 0.4, (1, 0): 0.2, (0, -1): 0.15, (-2, 3): 0.25}
    for (a, b), v in taps.items():
        h[a % N1, b % N2] = v
    # compact kernel with centre (c, c): tap (a, b) at [c + a, c + b]
    c = 3
    kc = np.zeros((2 * c + 1, 2 * c + 1))
    for (a, b), v in taps.items():
        kc[c + a, c + b] = v
    ref = scipy.ndimage.convolve(x, kc, mode="wrap", origin=0)
    assert np.allclose(model.conv_circ(x, h), ref, atol=1e-13)


def test_convolution_theorem_explicit_dft():
    """Section IV-A.1: H_{k,s} = F^H Lambda_{k,s} F, with Lambda the DFT of h.
    Checked with explicit DFT matrices, independent of numpy.fft."""
    rng = _rng(2)
    N1, N2 = 6, 8
    x = rng.standard_normal((N1, N2))
    h = rng.standard_normal((N1, N2))
    W1, W2 = _dft_matrix(N1), _dft_matrix(N2)
    lhs = W1 @ model.conv_circ(x, h) @ W2.T
    rhs = (W1 @ h @ W2.T) * (W1 @ x @ W2.T)
    assert np.allclose(lhs, rhs, atol=1e-11)


def test_adjoint_identity():
    """<Hx, y> = <x, H^T y> (transpose of the block matrix of Eq. forwardModel)."""
    x, psf = _small_problem(K=3, S=2, N1=16, N2=12)
    y = _rng(3).standard_normal((3, 16, 12))
    lhs = np.vdot(model.forward(x, psf), y)
    rhs = np.vdot(x, model.adjoint(y, psf))
    assert abs(lhs - rhs) <= 1e-13 * abs(lhs)


def test_dense_H_matches_operator():
    """The explicit BCCB block matrix reproduces the spatial operator."""
    x, psf = _small_problem(K=2, S=3, N1=6, N2=6)
    H = model.dense_H(psf)
    assert np.allclose(H @ x.ravel(), model.forward(x, psf).ravel(), atol=1e-13)
    y = _rng(4).standard_normal((2, 6, 6))
    assert np.allclose(H.T @ y.ravel(), model.adjoint(y, psf).ravel(), atol=1e-13)


def test_parseval_unitary_dft():
    """Unitary 2D DFT preserves energy (F_2D of Section IV-A.1 is unitary)."""
    x = _rng(5).standard_normal((8, 8))
    W = _dft_matrix(8) / math.sqrt(8)
    assert np.isclose(np.sum(x * x), np.sum(np.abs(W @ x @ W.T) ** 2), rtol=1e-13)


# ------------------------------------------------------------------ priors
def test_dct_matrix_matches_scipy_and_is_orthonormal():
    """The unitary T of Eq. analysis (DCT-II, orthonormal)."""
    for n in (1, 2, 8, 13):
        C = priors.dct_matrix(n)
        assert np.allclose(C @ C.T, np.eye(n), atol=1e-13)
        v = _rng(n).standard_normal(n)
        assert np.allclose(C @ v, scipy.fft.dct(v, type=2, norm="ortho"), atol=1e-13)


@pytest.mark.parametrize("kind", ["dct2d", "dct3d", "tv2d", "tv3d"])
def test_transform_adjoint(kind):
    T = priors.make_transform(kind, 3, 8, 6)
    x = _rng(6).standard_normal((3, 8, 6))
    w = _rng(7).standard_normal(T.shape)
    if kind == "tv3d":
        w[2, -1] = 0.0
    assert np.isclose(np.vdot(T.T(x), w), np.vdot(x, T.Tt(w)), rtol=1e-12)


def test_tv_symbol_matches_impulse_response():
    """T^T T of the anisotropic TV is circulant with DFT symbol
    (2 - 2cos w1) + (2 - 2cos w2) (used by the frequency-domain x-update)."""
    T = priors.TV2D(1, 8, 10)
    d = np.zeros((1, 8, 10))
    d[0, 0, 0] = 1.0
    imp = T.Tt(T.T(d))[0]
    W1, W2 = _dft_matrix(8), _dft_matrix(10)
    assert np.allclose(W1 @ imp @ W2.T, T.gram_symbol(8, 10), atol=1e-12)


def test_tv3d_band_laplacian():
    """The band-difference part of T^T T acts on per-band constants as the
    path-graph Laplacian."""
    S = 5
    T = priors.TV3D(S, 4, 4)
    c = _rng(8).standard_normal(S)
    x = np.broadcast_to(c[:, None, None], (S, 4, 4)).copy()
    out = T.Tt(T.T(x))[:, 0, 0]
    L = np.diag([1, 2, 2, 2, 1]) - np.diag(np.ones(4), 1) - np.diag(np.ones(4), -1)
    assert np.allclose(out, L @ c, atol=1e-13)
    assert np.allclose(T.band_laplacian(), L)


def test_soft_is_l1_prox_bruteforce():
    """Eq. solt_trans: soft(w, tau) = argmin_t tau|t| + 1/2 (t - w)^2."""
    grid = np.linspace(-4, 4, 160001)
    for w in (-2.3, -0.4, 0.0, 0.2, 1.7, 3.1):
        for tau in (0.0, 0.3, 1.0):
            f = tau * np.abs(grid) + 0.5 * (grid - w) ** 2
            assert abs(priors.soft(np.array(w), tau) - grid[np.argmin(f)]) < 1e-4
    # sign(0) = -1 is immaterial: soft(0) = 0
    assert priors.soft(np.array(0.0), 0.5) == 0.0


def test_patch_PtP_is_scaled_identity():
    """Eq. solx_synt: P^H P = t I; for Q = 8 and stride 4, t = 4."""
    P = priors.Patches(2, 16, 16, Q=8, st=4)
    n = 2 * 16 * 16
    M = np.zeros((n, n))
    e = np.zeros((2, 16, 16))
    for i in range(n):
        e.flat[i] = 1.0
        M[:, i] = P.adjoint(P.extract(e)).ravel()
        e.flat[i] = 0.0
    assert np.allclose(M, 4.0 * np.eye(n))
    assert P.c_P == 4.0
    # extract / adjoint are transposes of each other
    x = _rng(9).standard_normal((2, 16, 16))
    X = _rng(10).standard_normal((P.n, P.J))
    assert np.isclose(np.vdot(P.extract(x), X), np.vdot(x, P.adjoint(X)))


def test_patch_layout():
    """Element s*Q*Q + a*Q + b of patch (i, j) is x[s, i*st + a, j*st + b]."""
    S, N = 3, 16
    x = np.arange(S * N * N, dtype=float).reshape(S, N, N)
    P = priors.Patches(S, N, N, Q=8, st=4)
    X = P.extract(x)
    i, j, s, a, b = 3, 2, 1, 5, 7
    assert X[s * 64 + a * 8 + b, i * 4 + j] == x[s, (i * 4 + a) % N, (j * 4 + b) % N]


def test_conv_dict_spectra_and_adjoint():
    """Eq. conv_dic: D_m = F^H Theta_m F; synth/analysis are transposes."""
    filt = synth.random_unit_filters(_rng(11), 3, 5)
    cd = priors.ConvDict2D(filt, 2, 10, 12)
    z = _rng(12).standard_normal((3, 2, 10, 12))
    x = _rng(13).standard_normal((2, 10, 12))
    assert np.isclose(np.vdot(cd.synth(z), x), np.vdot(z, cd.analysis(x)))
    W1, W2 = _dft_matrix(10), _dft_matrix(12)
    lhs = W1 @ cd.synth(z)[1] @ W2.T
    rhs = sum((W1 @ cd.h[m] @ W2.T) * (W1 @ z[m, 1] @ W2.T) for m in range(3))
    assert np.allclose(lhs, rhs, atol=1e-10)


# ------------------------------------------------------------------ x-update
def test_recursive_block_inverse():
    """Eq. recinv (recursive 2x2 block inversion) equals the direct inverse."""
    rng = _rng(14)
    for S in (1, 2, 3, 4, 5, 8):
        A = rng.standard_normal((6, S, S)) + 1j * rng.standard_normal((6, S, S))
        psi = A @ np.conj(np.swapaxes(A, -1, -2)) + 0.1 * np.eye(S)
        inv = xupdate.recursive_block_inverse(psi)
        assert np.allclose(inv @ psi, np.eye(S)[None], atol=1e-10)


@pytest.mark.parametrize("kind", ["dct2d", "tv2d", "tv3d"])
def test_freq_solve_equals_dense_solve(kind):
    """Eq. solx_Trans_DFT equals Eq. solx_Trans (the dense normal equations)."""
    x, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=1)
    rho, beta = 0.05, 1.3
    T = priors.make_transform(kind, 2, 8, 8)
    dense = xupdate.DenseSolver(psf, beta, rho * xupdate.dense_TtT(T, 2, 8, 8),
                                annihilates_constants=(kind == "tv2d"))
    freq = xupdate.FreqSolver(psf, beta, rho, T.gram_symbol(8, 8),
                              T.band_laplacian() if kind == "tv3d" else None)
    y = model.forward(x, psf) + 0.01 * _rng(15).standard_normal((2, 8, 8))
    q = _rng(16).standard_normal(T.shape)
    if kind == "tv3d":
        q[2, -1] = 0
    extra = rho * T.Tt(q)
    xd = dense.solve(dense.data_term(y) + extra)
    xf = freq.solve(freq.data_term(y), extra)
    assert np.allclose(xd, xf, atol=1e-10 * np.max(np.abs(xd)))
    # and it is the minimum-norm minimiser: full pseudo-inverse of the normal matrix
    H = model.dense_H(psf)
    A = beta * H.T @ H + rho * xupdate.dense_TtT(T, 2, 8, 8)
    ref = np.linalg.pinv(A, rcond=1e-12, hermitian=True) @ (beta * H.T @ y.ravel() + extra.ravel())
    assert np.allclose(xd.ravel(), ref, atol=1e-9 * np.max(np.abs(ref)))


def test_tv2d_dc_block_is_singular_with_unit_sum_kernels():
    """With TV on every slice and unit-sum kernels the DC block is rank one
    (so the reading of a minimum-norm minimiser matters)."""
    _, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=2)
    lam = xupdate.psf_spectra(psf)
    T = priors.TV2D(2, 8, 8)
    psi = xupdate.gram_blocks(lam, 1.0, T.gram_symbol(8, 8), 0.01)
    ev = np.linalg.eigvalsh(psi[0, 0])
    assert ev[0] < 1e-12 * ev[-1]
    assert np.all(np.linalg.eigvalsh(psi[1:, :]) > 0)


def test_synthesis_freq_equals_dense():
    """Eq. solx_synt_DFT equals Eq. solx_synt."""
    x, psf = _small_problem(K=3, S=2, N1=8, N2=8, seed=3)
    beta, cP = 7.0, 4.0
    dense = xupdate.DenseSolver(psf, beta, cP * np.eye(2 * 64))
    freq = xupdate.FreqSolver(psf, beta, cP, np.ones((8, 8)))
    y = model.forward(x, psf)
    extra = _rng(17).standard_normal((2, 8, 8))
    assert np.allclose(dense.solve(dense.data_term(y) + extra),
                       freq.solve(freq.data_term(y), extra), atol=1e-11)


# ------------------------------------------------------------------ Algorithm 1
def test_dct_identity_blur_closed_form():
    """Algorithm 1 with H = I (delta kernels, K = S) solves
    min beta/2 ||y - x||^2 + lambda ||Cx||_1, whose minimiser is
    C^T soft(C y, lambda / beta) (orthonormal-basis denoising)."""
    S, N = 2, 8
    psf = np.zeros((S, S, N, N))
    for s in range(S):
        psf[s, s, 0, 0] = 1.0
    y = _rng(18).standard_normal((S, N, N))
    lam, beta, rho = 0.3, 1.0, 0.7
    alg = admm.AnalysisADMM(psf, "dct2d", lam, rho, beta, tier="freq")
    x, _, _ = alg.run(y, 400)
    T = priors.DCT2D(S, N, N)
    ref = T.Tt(priors.soft(T.T(y), lam / beta))
    assert np.allclose(x, ref, atol=1e-9)


def _qp_reference(y, psf, lam, beta, S, N):
    """min beta/2 ||y - H C^T c||^2 + lambda ||c||_1 as a bound-constrained
    smooth problem in (p, q >= 0), c = p - q, solved by L-BFGS-B."""
    H = model.dense_H(psf)
    C = priors.dct_matrix(N)
    Cst = np.kron(np.eye(S), np.kron(C, C))     # x = Cst^T c
    A = H @ Cst.T
    b = y.ravel()
    n = A.shape[1]

    def f(pq):
        c = pq[:n] - pq[n:]
        r = A @ c - b
        g = beta * (A.T @ r)
        val = 0.5 * beta * r @ r + lam * np.sum(pq)
        return val, np.concatenate([g + lam, -g + lam])

    res = scipy.optimize.minimize(f, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                                  bounds=[(0, None)] * (2 * n),
                                  options=dict(maxiter=20000, ftol=1e-16, gtol=1e-12,
                                               maxcor=50))
    c = res.x[:n] - res.x[n:]
    return (Cst.T @ c).reshape(S, N, N), res.fun


def test_dct_admm_matches_bruteforce_qp():
    """Algorithm 1 (DCT-l1) converges to the minimiser found by a generic
    bound-constrained optimiser."""
    S, N = 2, 6
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=4)
    y = model.forward(x0, psf) + 0.02 * _rng(19).standard_normal((2, N, N))
    lam, beta, rho = 0.02, 1.0, 0.2
    alg = admm.AnalysisADMM(psf, "dct2d", lam, rho, beta, tier="dense")
    x, t, u = alg.run(y, 3000)
    xr, fr = _qp_reference(y, psf, lam, beta, S, N)
    f = admm.analysis_objective(x, y, psf, alg.T, lam, beta)
    assert f <= fr + 1e-9 * abs(fr)
    assert np.allclose(x, xr, atol=2e-5)


@pytest.mark.parametrize("kind", ["dct2d", "tv2d", "tv3d"])
def test_admm_kkt_vanishes(kind):
    """At convergence the KKT residuals of the split problem vanish and the
    running minimum of the objective is non-increasing."""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=5)
    y = model.forward(x0, psf) + 0.01 * _rng(20).standard_normal((2, N, N))
    alg = admm.AnalysisADMM(psf, kind, lam=0.01, rho=0.1, beta=1.0, tier="dense")
    fs = []
    alg_cb = lambda it, x, t, u: fs.append(
        admm.analysis_objective(x, y, psf, alg.T, alg.lam, alg.beta))
    x, t, u = alg.run(y, 4000, callback=alg_cb)
    r1, r2, r3 = alg.kkt(y, x, t, u)
    assert max(r1, r2, r3) < 1e-9
    assert fs[-1] < fs[0]
    run_min = np.minimum.accumulate(fs)
    assert np.all(np.diff(run_min) <= 0)


def test_admm_lambda_zero_gives_least_squares():
    """With lambda = 0 the fixed point is the (minimum-norm) least-squares
    solution (beta H^T H)^+ beta H^T y."""
    S, N = 2, 6
    rng = _rng(6)
    psf = synth.gaussian_psfs(rng, 3, S, N, N, sigma_range=(0.3, 0.7))
    x0 = rng.uniform(0, 1, (S, N, N))
    y = model.forward(x0, psf) + 0.01 * _rng(21).standard_normal((3, N, N))
    alg = admm.AnalysisADMM(psf, "dct2d", lam=0.0, rho=0.05, beta=1.0, tier="dense")
    x, _, _ = alg.run(y, 3000)
    H = model.dense_H(psf)
    ref = np.linalg.pinv(H.T @ H, rcond=1e-13, hermitian=True) @ (H.T @ y.ravel())
    assert np.allclose(x.ravel(), ref, atol=1e-7)


def test_dense_and_freq_tiers_agree_over_iterations():
    """Tier D and tier F implement the same iteration (TV2D, singular DC)."""
    x0, psf = _small_problem(K=2, S=2, N1=16, N2=16, seed=7)
    y = model.forward(x0, psf) + 0.01 * _rng(22).standard_normal((2, 16, 16))
    a = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="dense").run(y, 30)[0]
    b = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="freq").run(y, 30)[0]
    assert admm.rel_l2(b, a) < 1e-10


# ------------------------------------------------------------------ Algorithm 2
def test_patch_z_update_is_subproblem_minimiser():
    """Eq. solz_patch2 minimises Eq. iterd_ADMM2 for the patch prior: the
    gradient D^T (D z - P x) + rho (z - t + u) vanishes."""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=8)
    D = synth.random_unit_atoms(_rng(23), 4 * 4 * S, 40)
    alg = admm.PatchADMM(psf, D, Q=4, stride=2, lam=1e-3, rho=0.3, beta=10.0)
    t = _rng(24).standard_normal((40, alg.P.J))
    u = _rng(25).standard_normal((40, alg.P.J))
    z = alg.z_update(x0, t, u)
    g = D.T @ (D @ z - alg.P.extract(x0)) + 0.3 * (z - t + u)
    assert np.max(np.abs(g)) < 1e-10


def test_patch_x_update_is_subproblem_minimiser():
    """Eq. solx_synt minimises Eq. iterd_ADMM1 (squared norms): gradient
    beta H^T (Hx - y) + P^T (P x - D z) vanishes."""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=9)
    D = synth.random_unit_atoms(_rng(26), 4 * 4 * S, 40)
    y = model.forward(x0, psf)
    for tier in ("dense", "freq"):
        alg = admm.PatchADMM(psf, D, Q=4, stride=2, lam=1e-3, rho=0.3, beta=10.0, tier=tier)
        z = _rng(27).standard_normal((40, alg.P.J))
        x = alg.x_update(alg.solver.data_term(y), z)
        g = 10.0 * model.adjoint(model.forward(x, psf) - y, psf) \
            + alg.P.adjoint(alg.P.extract(x) - D @ z)
        assert np.max(np.abs(g)) < 1e-9


def test_patch_admm_kkt():
    """Algorithm 2 (patch prior) approaches a KKT point of the synthesis problem:
    z = t, stationarity in x and z, and the prox fixed point. (ADMM converges
    sublinearly here; the residuals are checked at a level where a dropped or
    mis-signed term would show as an O(1) residual.)"""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=10)
    y = model.forward(x0, psf) + 0.01 * _rng(28).standard_normal((2, N, N))
    D = synth.random_unit_atoms(_rng(29), 4 * 4 * S, 32)
    lam, rho, beta = 1e-2, 1.0, 5.0
    alg = admm.PatchADMM(psf, D, Q=4, stride=2, lam=lam, rho=rho, beta=beta)
    x, z, t, u = alg.run(y, 3000)
    assert np.linalg.norm(z - t) < 1e-6 * np.linalg.norm(z)
    scale = np.max(np.abs(beta * model.adjoint(y, psf)))
    gx = beta * model.adjoint(model.forward(x, psf) - y, psf) \
        + alg.P.adjoint(alg.P.extract(x) - D @ z)
    assert np.max(np.abs(gx)) < 1e-5 * scale
    gz = D.T @ (D @ z - alg.P.extract(x)) + rho * u
    assert np.max(np.abs(gz)) < 5e-5 * np.max(np.abs(D.T @ alg.P.extract(x)))
    assert np.linalg.norm(t - priors.soft(t + u, lam / rho)) < 1e-6 * np.linalg.norm(t)


def _patch_dl(seed, S=2, N=8, A=24, sigma=0.7):
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=seed)
    D = synth.random_unit_atoms(_rng(seed + 200), 4 * 4 * S, A)
    D = D / np.linalg.norm(D)
    alg = admm.PatchADMM(psf, D, Q=4, stride=2, lam=1e-3, rho=0.3, beta=10.0,
                         dict_update=True, sigma=sigma)
    return x0, psf, alg


def test_patch_dictionary_d_update_minimises_its_objective():
    """Eq. ADMM0: the D-update minimises 1/2 ||D Z - X||_F^2 + sigma/2
    ||D - G + E||_F^2 (checked against a least-squares solve of the stacked
    system [Z^T; sqrt(sigma) I] D^T = [X^T; sqrt(sigma) (G - E)^T] and by
    random perturbations)."""
    x0, psf, alg = _patch_dl(30)
    A, n = alg.D.shape[1], alg.D.shape[0]
    alg.g = _rng(31).standard_normal((n, A))
    alg.e = 0.3 * _rng(32).standard_normal((n, A))
    X = _rng(33).standard_normal((n, 50))
    Z = _rng(34).standard_normal((A, 50))
    D = alg.d_update_patches(X, Z)
    sq = math.sqrt(alg.sigma)
    lhs = np.vstack([Z.T, sq * np.eye(A)])
    rhs = np.vstack([X.T, sq * (alg.g - alg.e).T])
    ref = np.linalg.lstsq(lhs, rhs, rcond=None)[0].T
    assert np.max(np.abs(D - ref)) < 1e-10

    def f(Dm):
        return 0.5 * np.sum((Dm @ Z - X) ** 2) + 0.5 * alg.sigma * np.sum((Dm - alg.g + alg.e) ** 2)
    f0 = f(D)
    for i in range(5):
        assert f(D + 1e-3 * _rng(35 + i).standard_normal(D.shape)) > f0


def test_patch_dictionary_d_update_recovers_a_consistent_dictionary():
    """With X = D* Z exactly and a vanishing sigma, Eq. sold_patch returns
    D* (Z has full row rank)."""
    x0, psf, alg = _patch_dl(40, sigma=1e-12)
    n, A = alg.D.shape
    Dstar = _rng(41).standard_normal((n, A))
    Z = _rng(42).standard_normal((A, 200))
    D = alg.d_update_patches(Dstar @ Z, Z)
    assert np.max(np.abs(D - Dstar)) < 1e-8


def test_patch_dictionary_g_update_is_the_projection():
    """Eq. ADMM1: G is the point of the unit Frobenius sphere nearest to
    D + E: unit norm, a positive multiple of D + E, and no random unit
    matrix is closer."""
    x0, psf, alg = _patch_dl(50)
    n, A = alg.D.shape
    d = _rng(51).standard_normal((n, A))
    alg.e = _rng(52).standard_normal((n, A))
    g = alg.g_update(d)
    w = d + alg.e
    assert abs(np.linalg.norm(g) - 1.0) < 1e-12
    c = np.sum(g * w) / np.sum(w * w)
    assert c > 0 and np.max(np.abs(g - c * w)) < 1e-14
    dist = np.linalg.norm(g - w)
    for i in range(20):
        q = _rng(53 + i).standard_normal((n, A))
        assert np.linalg.norm(q / np.linalg.norm(q) - w) > dist


def test_patch_dictionary_update_with_huge_sigma_keeps_the_dictionary():
    """sigma -> infinity pins D to G - E = G; with ||G||_F = 1 the
    projection keeps it, so the run equals the fixed-dictionary run; a
    finite sigma moves the dictionary and keeps ||G||_F = 1."""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=60)
    y = model.forward(x0, psf) + 0.01 * _rng(61).standard_normal((2, N, N))
    D = synth.random_unit_atoms(_rng(62), 4 * 4 * S, 24)
    D = D / np.linalg.norm(D)
    kw = dict(Q=4, stride=2, lam=1e-3, rho=0.3, beta=10.0)
    a = admm.PatchADMM(psf, D, **kw).run(y, 10)
    b = admm.PatchADMM(psf, D, dict_update=True, sigma=1e12, **kw).run(y, 10)
    assert admm.rel_l2(b[0], a[0]) < 1e-8
    alg = admm.PatchADMM(psf, D, dict_update=True, sigma=1.0, **kw)
    c = alg.run(y, 10)
    assert admm.rel_l2(c[0], a[0]) > 1e-4
    assert abs(np.linalg.norm(alg.g) - 1.0) < 1e-12
    assert np.max(np.abs(alg.D - alg.g)) == 0.0


def test_patch_dictionary_learning_lowers_the_patch_fit():
    """With E = 0, Eq. ADMM0 minimises fit(D) + sigma/2 ||D - G||_F^2 with
    fit(D) = 1/2 ||D Z - X||_F^2, whose value at D = G is fit(G): the D-step
    satisfies fit(D) + sigma/2 ||D - G||_F^2 <= fit(G)."""
    x0, psf, alg = _patch_dl(70, sigma=0.05)
    n, A = alg.D.shape
    X = alg.P.extract(x0)
    Z = _rng(71).standard_normal((A, alg.P.J)) * 0.1
    D = alg.d_update_patches(X, Z)
    fit = lambda Dm: 0.5 * np.sum((Dm @ Z - X) ** 2)
    assert fit(D) + 0.5 * alg.sigma * np.sum((D - alg.g) ** 2) <= fit(alg.g) + 1e-12


def test_sherman_morrison_equals_dense_solve():
    """Eq. solz_DFT_SM equals a dense solve of (rho I + Theta^H Theta) v = c."""
    rng = _rng(30)
    M = 7
    theta = rng.standard_normal((M, 5)) + 1j * rng.standard_normal((M, 5))
    c = rng.standard_normal((M, 5)) + 1j * rng.standard_normal((M, 5))
    for rho in (1e-4, 0.3, 10.0):
        v = admm.sherman_morrison(theta, c, rho)
        for f in range(5):
            a = np.conj(theta[:, f])
            A = rho * np.eye(M) + np.outer(a, np.conj(a))
            assert np.allclose(v[:, f], np.linalg.solve(A, c[:, f]), rtol=1e-9, atol=1e-12)


def test_conv_z_update_is_subproblem_minimiser():
    """Eq. solz / solz_DFT: the gradient D~^T (D~ z - x) + rho (z - t + u)
    vanishes (checked with the spatial-domain dictionary operators)."""
    S, N, M = 2, 12, 3
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=11)
    filt = synth.random_unit_filters(_rng(31), M, 5)
    alg = admm.ConvADMM(psf, filt, lam=1e-3, rho=0.2, beta=5.0, tier="freq")
    t = _rng(32).standard_normal((M, S, N, N))
    u = _rng(33).standard_normal((M, S, N, N))
    z = alg.z_update(x0, t, u)
    g = alg.cd.analysis(alg.cd.synth(z) - x0) + 0.2 * (z - t + u)
    assert np.max(np.abs(g)) < 1e-10


def test_conv_admm_tiers_agree_and_converge():
    """Algorithm 2 (conv prior): the spatial (dense) and frequency tiers run
    the same iteration, and the iteration reaches z = t."""
    S, N, M = 2, 8, 3
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=12)
    y = model.forward(x0, psf) + 0.01 * _rng(34).standard_normal((2, N, N))
    filt = synth.random_unit_filters(_rng(35), M, 3)
    a = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="dense").run(y, 20)
    b = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq").run(y, 20)
    assert admm.rel_l2(b[0], a[0]) < 1e-10
    x, z, t, u = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq").run(y, 2000)
    assert np.linalg.norm(z - t) < 2e-6 * np.linalg.norm(z)


def _filters3(rng, M, S, L):
    f = rng.standard_normal((M, S, L, L))
    return f / np.linalg.norm(f.reshape(M, -1), axis=1)[:, None, None, None]


def test_conv3d_synthesis_theorem_and_adjoint():
    """3D dictionary: the spatial 3D circular convolutions equal the 3D-DFT
    products (convolution theorem along the bands too), and the correlation
    is their adjoint."""
    S, N, M, L = 3, 8, 2, 3
    cd = priors.ConvDict3D(_filters3(_rng(70), M, S, L), S, N, N)
    z = _rng(71).standard_normal((M, S, N, N))
    y = _rng(72).standard_normal((S, N, N))
    ref = cd.synth(z)
    via_fft = np.real(np.fft.ifftn(np.sum(cd.spectra() * np.fft.fftn(z, axes=(1, 2, 3)), axis=0)))
    assert np.max(np.abs(via_fft - ref)) < 1e-12
    # a single tap at band offset 1 shifts the bands by one (circularly)
    f = np.zeros((1, S, 1, 1))
    f[0, 1, 0, 0] = 1.0
    shift = priors.ConvDict3D(f, S, N, N).synth(z[:1])
    assert np.allclose(shift, np.roll(z[0], 1, axis=0), atol=1e-14)
    assert abs(np.vdot(ref, y) - np.vdot(z, cd.analysis(y))) < 1e-10 * abs(np.vdot(ref, y))


def test_conv3d_z_update_is_subproblem_minimiser():
    """3D codes: the gradient D~^T (D~ z - x) + rho (z - t + u) vanishes at
    the frequency-domain z-update (spatial-domain operators)."""
    S, N, M = 3, 10, 2
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=13)
    alg = admm.ConvADMM(psf, _filters3(_rng(73), M, S, 3), lam=1e-3, rho=0.2, beta=5.0,
                        tier="freq", dims=3)
    t = _rng(74).standard_normal((M, S, N, N))
    u = _rng(75).standard_normal((M, S, N, N))
    z = alg.z_update(x0, t, u)
    g = alg.cd.analysis(alg.cd.synth(z) - x0) + 0.2 * (z - t + u)
    assert np.max(np.abs(g)) < 1e-10


def test_conv3d_single_band_is_the_2d_dictionary():
    """With S = 1 the 3D dictionary is the 2D one: the two runs coincide."""
    N, M = 8, 3
    x0, psf = _small_problem(K=1, S=1, N1=N, N2=N, seed=14)
    y = model.forward(x0, psf) + 0.01 * _rng(76).standard_normal((1, N, N))
    f2 = synth.random_unit_filters(_rng(77), M, 3)
    a = admm.ConvADMM(psf, f2, 1e-3, 0.5, 10.0, tier="freq").run(y, 15)
    b = admm.ConvADMM(psf, f2[:, None], 1e-3, 0.5, 10.0, tier="freq", dims=3).run(y, 15)
    assert admm.rel_l2(b[0], a[0]) < 1e-12


def test_conv3d_admm_tiers_agree_and_converge():
    """Algorithm 2 with 3D filters: the spatial (dense) and frequency tiers
    run the same iteration, and the iteration reaches z = t."""
    S, N, M = 2, 8, 2
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=15)
    y = model.forward(x0, psf) + 0.01 * _rng(78).standard_normal((2, N, N))
    filt = _filters3(_rng(79), M, S, 3)
    a = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="dense", dims=3).run(y, 20)
    b = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", dims=3).run(y, 20)
    assert admm.rel_l2(b[0], a[0]) < 1e-10
    x, z, t, u = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", dims=3).run(y, 2000)
    assert np.linalg.norm(z - t) < 2e-6 * np.linalg.norm(z)


def _conv3_brute(z, h):
    """sum over the nonzero taps of h of h[s', a, b] z[s - s', n1 - a, n2 - b]
    (circular), by shifts: no FFT."""
    out = np.zeros_like(z)
    for (sp, a, b) in zip(*np.nonzero(h)):
        out += h[sp, a, b] * np.roll(z, (sp, a, b), axis=(0, 1, 2))
    return out


def _corr3_brute(y, h):
    out = np.zeros_like(y)
    for (sp, a, b) in zip(*np.nonzero(h)):
        out += h[sp, a, b] * np.roll(y, (-sp, -a, -b), axis=(0, 1, 2))
    return out


def test_conv3d_dictionary_d_update_solves_its_normal_equation():
    """Eq. sold_3D: (sigma I + Z^H Z) d = Z^H x + sigma (g - e), with Z_m the
    3D circular convolution by the code z_m (brute-force shifts)."""
    S, N, M = 2, 6, 2
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=16)
    alg = admm.ConvADMM(psf, _filters3(_rng(80), M, S, 3), 1e-3, 0.5, 10.0, tier="freq",
                        dims=3, dict_update=True, sigma=0.7)
    alg.e = 0.1 * _rng(81).standard_normal(alg.e.shape)
    z = _rng(82).standard_normal((M, S, N, N))
    d = alg.d_update(x0, z)
    zd = sum(_conv3_brute(d[m], z[m]) for m in range(M))
    for m in range(M):
        res = 0.7 * d[m] + _corr3_brute(zd - x0, z[m]) - 0.7 * (alg.g[m] - alg.e[m])
        assert np.max(np.abs(res)) < 1e-10


def test_conv3d_dictionary_g_update_is_the_projection():
    """Eq. g_admm: g_m is d_m + e_m cropped to the L x L x S support and
    scaled to unit norm (the nearest point of C_d)."""
    S, N, M, L = 2, 8, 3, 3
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=17)
    alg = admm.ConvADMM(psf, _filters3(_rng(83), M, S, L), 1e-3, 0.5, 10.0, tier="freq",
                        dims=3, dict_update=True)
    d = _rng(84).standard_normal((M, S, N, N))
    alg.e = _rng(85).standard_normal((M, S, N, N))
    g = alg.g_update(d)
    mask = np.zeros((N, N), bool)
    for a in range(L):
        for b in range(L):
            mask[(a - L // 2) % N, (b - L // 2) % N] = True
    for m in range(M):
        assert abs(np.linalg.norm(g[m]) - 1.0) < 1e-12
        assert np.all(g[m][:, ~mask] == 0.0)
        w = (d[m] + alg.e[m])[:, mask]
        assert np.allclose(g[m][:, mask], w / np.linalg.norm(w), atol=1e-14)


def test_conv3d_dictionary_update_with_huge_sigma_keeps_the_dictionary():
    """sigma -> infinity pins d to g - e = g, so the run equals the
    fixed-dictionary run (the updated filters feed the next x- and
    z-updates)."""
    S, N, M = 2, 8, 2
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=18)
    y = model.forward(x0, psf) + 0.01 * _rng(86).standard_normal((2, N, N))
    filt = _filters3(_rng(87), M, S, 3)
    a = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", dims=3).run(y, 10)
    alg = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", dims=3, dict_update=True,
                        sigma=1e12)
    b = alg.run(y, 10)
    assert admm.rel_l2(b[0], a[0]) < 1e-8
    alg2 = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", dims=3, dict_update=True,
                         sigma=1.0)
    c = alg2.run(y, 10)
    assert admm.rel_l2(c[0], a[0]) > 1e-4          # a finite sigma does move the dictionary
    assert np.allclose(np.linalg.norm(alg2.g.reshape(M, -1), axis=1), 1.0, atol=1e-12)


def test_conv2d_dictionary_d_update_solves_its_normal_equation():
    """2D form (common filters): (sigma I + sum_s Z_s^H Z_s) d = sum_s
    Z_s^H x_s + sigma (g - e), Z_{m,s} the 2D circular convolution by the
    code z_{m,s} (shifts, no FFT)."""
    S, N, M = 3, 6, 2
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=19)
    alg = admm.ConvADMM(psf, synth.random_unit_filters(_rng(88), M, 3), 1e-3, 0.5, 10.0,
                        tier="freq", dict_update=True, sigma=0.7)
    alg.e = 0.1 * _rng(89).standard_normal(alg.e.shape)
    z = _rng(90).standard_normal((M, S, N, N))
    d = alg.d_update(x0, z)
    resid = [sum(model.conv_circ(d[m], z[m, s]) for m in range(M)) - x0[s] for s in range(S)]
    for m in range(M):
        g = 0.7 * (d[m] - alg.g[m] + alg.e[m])
        g = g + sum(model.corr_circ(resid[s], z[m, s]) for s in range(S))
        assert np.max(np.abs(g)) < 1e-10


def test_dictionary_learning_single_plane_3d_equals_2d():
    """With S = 1 the 3D and 2D dictionary updates coincide."""
    N, M = 8, 3
    x0, psf = _small_problem(K=1, S=1, N1=N, N2=N, seed=20)
    y = model.forward(x0, psf) + 0.01 * _rng(91).standard_normal((1, N, N))
    f2 = synth.random_unit_filters(_rng(92), M, 3)
    a = admm.ConvADMM(psf, f2, 1e-3, 0.5, 10.0, tier="freq", dict_update=True, sigma=2.0)
    b = admm.ConvADMM(psf, f2[:, None], 1e-3, 0.5, 10.0, tier="freq", dims=3,
                      dict_update=True, sigma=2.0)
    ra, rb = a.run(y, 12), b.run(y, 12)
    assert admm.rel_l2(rb[0], ra[0]) < 1e-12
    assert np.max(np.abs(b.g[:, 0] - a.g)) < 1e-12


def test_tikhonov_symbol_closed_form():
    """sum_i |DFT(r_i)|^2 of the two circular forward differences is
    (2 - 2 cos w1) + (2 - 2 cos w2)."""
    N1, N2 = 6, 10
    w1 = 2 * np.pi * np.arange(N1)[:, None] / N1
    w2 = 2 * np.pi * np.arange(N2)[None, :] / N2
    ref = (2 - 2 * np.cos(w1)) + (2 - 2 * np.cos(w2))
    assert np.allclose(priors.tikhonov_symbol(N1, N2), ref, atol=1e-13)
    # the kernels are forward differences: r_1 * z = z[n1 + 1] - z[n1]
    z = _rng(60).standard_normal((N1, N2))
    r1, r2 = priors.gradient_filters_2d(N1, N2)
    assert np.allclose(model.conv_circ(z, r1), np.roll(z, -1, axis=0) - z, atol=1e-12)
    assert np.allclose(model.conv_circ(z, r2), np.roll(z, -1, axis=1) - z, atol=1e-12)


def test_sherman_morrison_frequency_dependent_diagonal():
    """(c(w) I + a a^H) v = rhs with a diagonal that varies with frequency."""
    rng = _rng(61)
    M = 5
    theta = rng.standard_normal((M, 6)) + 1j * rng.standard_normal((M, 6))
    rhs = rng.standard_normal((M, 6)) + 1j * rng.standard_normal((M, 6))
    cdiag = rng.uniform(1e-4, 3.0, 6)
    v = admm.sherman_morrison(theta, rhs, cdiag)
    for f in range(6):
        a = np.conj(theta[:, f])
        A = cdiag[f] * np.eye(M) + np.outer(a, np.conj(a))
        assert np.allclose(v[:, f], np.linalg.solve(A, rhs[:, f]), rtol=1e-9, atol=1e-12)


def test_conv_tikhonov_z_update_is_subproblem_minimiser():
    """With the gradient regulariser the z-update minimises
    1/2 ||D~ z - x||^2 + mu/2 sum_i ||r_i * z||^2 + rho/2 ||z - t + u||^2:
    the gradient D~^T (D~ z - x) + mu sum_i R_i^T R_i z + rho (z - t + u)
    vanishes (R_i^T R_i z = 2 z - z[n - e_i] - z[n + e_i], spatial)."""
    S, N, M = 2, 12, 3
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=13)
    filt = synth.random_unit_filters(_rng(62), M, 5)
    mu, rho = 0.3, 0.2
    alg = admm.ConvADMM(psf, filt, lam=1e-3, rho=rho, beta=5.0, tier="freq", mu=mu)
    t = _rng(63).standard_normal((M, S, N, N))
    u = _rng(64).standard_normal((M, S, N, N))
    z = alg.z_update(x0, t, u)
    lap = sum(2 * z - np.roll(z, 1, axis=ax) - np.roll(z, -1, axis=ax) for ax in (2, 3))
    g = alg.cd.analysis(alg.cd.synth(z) - x0) + mu * lap + rho * (z - t + u)
    assert np.max(np.abs(g)) < 1e-10
    # and it differs from the unregularised update
    z0 = admm.ConvADMM(psf, filt, lam=1e-3, rho=rho, beta=5.0, tier="freq").z_update(x0, t, u)
    assert np.linalg.norm(z - z0) > 1e-2 * np.linalg.norm(z0)


def test_conv_tikhonov_admm_converges():
    """Algorithm 2 with the gradient regulariser reaches z = t."""
    S, N, M = 2, 8, 3
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=14)
    y = model.forward(x0, psf) + 0.01 * _rng(65).standard_normal((2, N, N))
    filt = synth.random_unit_filters(_rng(66), M, 3)
    x, z, t, u = admm.ConvADMM(psf, filt, 1e-3, 0.5, 10.0, tier="freq", mu=0.1).run(y, 2000)
    assert np.linalg.norm(z - t) < 2e-6 * np.linalg.norm(z)


# ---------------------------------------------------------------- adaptive rho (Eq. paramS)
def test_adaptive_without_changes_equals_run():
    """With the balance factor so large that rho never changes and no
    stopping, the adaptive run is Algorithm 1 with fixed rho."""
    x0, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=40)
    y = model.forward(x0, psf) + 0.01 * _rng(70).standard_normal((2, 8, 8))
    for kind in ("dct2d", "tv2d", "tv3d"):
        alg = admm.AnalysisADMM(psf, kind, 1e-2, 0.1, 1.0, tier="freq")
        xa, info = alg.run_adaptive(y, 30, mu=1e30, every=1, tol=0.0)
        xr = admm.AnalysisADMM(psf, kind, 1e-2, 0.1, 1.0, tier="freq").run(y, 30)[0]
        assert info["iters"] == 30 and info["rhos"] == [0.1] * 30   # checks at 1 .. 29
        assert np.array_equal(xa, xr)


def test_adaptive_rescaling_keeps_the_fixed_point():
    """At a fixed point of Algorithm 1 with penalty rho, switching to rho' with
    u rescaled by rho / rho' leaves the iterate where it is (the scaled dual
    of rho' is u rho / rho'); the opposite rescaling moves it."""
    x0, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=41)
    y = model.forward(x0, psf) + 0.01 * _rng(71).standard_normal((2, 8, 8))
    lam, rho = 1e-2, 0.5
    x, t, u = admm.AnalysisADMM(psf, "dct2d", lam, rho, 1.0, tier="freq").run(y, 3000)
    rho2 = 2.0 * rho
    nxt = admm.AnalysisADMM(psf, "dct2d", lam, rho2, 1.0, tier="freq")
    x_ok = nxt.run(y, 1, state=(t, u * rho / rho2))[0]
    x_bad = nxt.run(y, 1, state=(t, u * rho2 / rho))[0]
    assert np.linalg.norm(x_ok - x) < 1e-9 * np.linalg.norm(x)
    assert np.linalg.norm(x_bad - x) > 1e-4 * np.linalg.norm(x)


def test_adaptive_reaches_the_minimiser_and_moves_rho():
    """From a poor starting penalty the adaptive run changes rho and stops
    at the DCT-l1 minimiser (unique), the same point fixed-rho ADMM reaches."""
    x0, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=42)
    y = model.forward(x0, psf) + 0.01 * _rng(72).standard_normal((2, 8, 8))
    lam = 1e-2
    ref = admm.AnalysisADMM(psf, "dct2d", lam, 0.1, 1.0, tier="freq").run(y, 20000)[0]
    for rho0, first in ((1e-5, "up"), (1e3, "down")):
        alg = admm.AnalysisADMM(psf, "dct2d", lam, rho0, 1.0, tier="freq")
        x, info = alg.run_adaptive(y, 20000, every=1, tol=1e-11)
        assert info["iters"] < 20000
        changes = [b / a for a, b in zip(info["rhos"], info["rhos"][1:]) if b != a]
        assert changes and changes[0] == (2.0 if first == "up" else 0.5)
        assert np.linalg.norm(x - ref) < 1e-6 * np.linalg.norm(ref)
        assert alg.rho == rho0          # the object is left with its own rho


def test_adaptive_stops_at_first_check_below_tolerance():
    x0, psf = _small_problem(K=2, S=2, N1=8, N2=8, seed=43)
    y = model.forward(x0, psf) + 0.01 * _rng(73).standard_normal((2, 8, 8))
    alg = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="freq")
    x, info = alg.run_adaptive(y, 5000, every=5, tol=1e-3)
    assert info["iters"] % 5 == 0 and info["iters"] < 5000
    assert info["rel_change"] < 1e-3
    # one check earlier the change was still above the tolerance
    x2, info2 = admm.AnalysisADMM(psf, "tv2d", 1e-3, 1e-2, 1.0, tier="freq").run_adaptive(
        y, info["iters"] - 4, every=5, tol=0.0)   # its last check is at iters - 5
    assert info2["rel_change"] >= 1e-3


# ---------------------------------------------------------------- 3D DCT prior
def test_dct3d_matches_scipy_dctn_and_is_orthonormal():
    """T of the 3D DCT prior is scipy's orthonormal DCT-II over all three axes."""
    S, N1, N2 = 5, 6, 4
    T = priors.DCT3D(S, N1, N2)
    x = _rng(80).standard_normal((S, N1, N2))
    assert np.allclose(T.T(x)[0], scipy.fft.dctn(x, type=2, norm="ortho"), atol=1e-12)
    assert np.allclose(T.Tt(T.T(x)), x, atol=1e-12)
    assert np.isclose(np.linalg.norm(T.T(x)), np.linalg.norm(x), rtol=1e-13)


def test_dct3d_identity_blur_closed_form():
    """With H = I the DCT3D-l1 problem is orthonormal-basis denoising: the
    minimiser is T^T soft(T y, lambda / beta), which differs from the
    per-slice (2D) answer when S > 1."""
    S, N = 3, 8
    psf = np.zeros((S, S, N, N))
    for s in range(S):
        psf[s, s, 0, 0] = 1.0
    y = _rng(81).standard_normal((S, N, N))
    lam, beta, rho = 0.3, 1.0, 0.7
    x, _, _ = admm.AnalysisADMM(psf, "dct3d", lam, rho, beta, tier="freq").run(y, 400)
    T = priors.DCT3D(S, N, N)
    ref = T.Tt(priors.soft(T.T(y), lam / beta))
    assert np.allclose(x, ref, atol=1e-9)
    x2 = priors.DCT2D(S, N, N)
    ref2 = x2.Tt(priors.soft(x2.T(y), lam / beta))
    assert np.linalg.norm(ref - ref2) > 1e-2 * np.linalg.norm(ref)


def test_dct3d_admm_kkt():
    x0, psf = _small_problem(K=3, S=3, N1=8, N2=8, seed=44)
    y = model.forward(x0, psf) + 0.01 * _rng(82).standard_normal((3, 8, 8))
    alg = admm.AnalysisADMM(psf, "dct3d", 1e-2, 0.2, 1.0, tier="freq")
    x, t, u = alg.run(y, 3000)
    r1, r2, r3 = alg.kkt(y, x, t, u)
    assert r1 < 1e-8 and r2 < 1e-8 and r3 < 1e-8


# ---------------------------------------------------------------- isotropic TV (T = I, Chambolle)
def test_symmlet8_filter_is_orthonormal_with_eight_vanishing_moments():
    """The Symmlet-8 scaling filter (Section V-A's wavelet): sum sqrt(2), unit
    energy, orthogonal to its even shifts; its wavelet filter annihilates
    polynomials of degree < 8 and not degree 8; the filter is not the
    minimum-phase one (zeros on both sides of the unit circle: the
    least-asymmetric choice of the family)."""
    h = priors.SYM8
    assert len(h) == 16
    assert abs(h.sum() - math.sqrt(2.0)) < 1e-12
    assert abs(np.dot(h, h) - 1.0) < 1e-12
    for m in range(1, 8):
        assert abs(np.dot(h[:-2 * m], h[2 * m:])) < 1e-12
    g = priors.qmf_highpass(h)
    t = np.arange(16.0)
    for p in range(8):
        assert abs(np.sum(g * t ** p)) < 1e-8 * np.sum(np.abs(g) * t ** p)
    assert abs(np.sum(g * t ** 8)) > 1e3
    r = np.abs(np.roots(h))
    assert np.any(r < 0.9) and np.any(r > 1.1)


def test_dwt1_equals_the_explicit_analysis_matrix():
    """One periodized DWT level equals the product with the matrix whose row k
    holds h[t] at column (2k + t) mod N (low-pass half) and g[t] likewise
    (high-pass half), built entry by entry; that matrix is orthogonal."""
    N = 32
    h = priors.SYM8
    g = priors.qmf_highpass(h)
    W = np.zeros((N, N))
    for k in range(N // 2):
        for t in range(16):
            W[k, (2 * k + t) % N] += h[t]
            W[N // 2 + k, (2 * k + t) % N] += g[t]
    assert np.allclose(W @ W.T, np.eye(N), atol=1e-12)
    x = _rng(120).standard_normal((3, N))
    assert np.allclose(priors.dwt1(x, h, axis=1), x @ W.T, atol=1e-13)
    assert np.allclose(priors.idwt1(x @ W.T, h, axis=1), x, atol=1e-12)
    # N smaller than the filter: the taps wrap around more than once
    N = 8
    W = np.zeros((N, N))
    for k in range(N // 2):
        for t in range(16):
            W[k, (2 * k + t) % N] += h[t]
            W[N // 2 + k, (2 * k + t) % N] += g[t]
    x = _rng(121).standard_normal((2, N))
    assert np.allclose(priors.dwt1(x, h, axis=1), x @ W.T, atol=1e-13)


def test_wavelet_dct_is_orthonormal_and_maps_constants_to_one_coefficient():
    """T = (2D Symmlet-8, 3 levels per slice) then DCT along the bands is
    orthonormal (T^T T = I, T T^T = I on random data); a constant cube c
    goes to the single coefficient sqrt(S) c 2^levels at the first band-DCT
    index and the top-left corner (sum h = sqrt(2) per axis and level, zero
    wavelet moment)."""
    S, N1, N2 = 3, 32, 16
    T = priors.WaveletDCT(S, N1, N2, levels=3)
    x = _rng(122).standard_normal((S, N1, N2))
    w = T.T(x)
    assert abs(np.linalg.norm(w) - np.linalg.norm(x)) < 1e-12 * np.linalg.norm(x)
    assert np.allclose(T.Tt(w), x, atol=1e-12)
    c = _rng(123).standard_normal((1, S, N1, N2))
    assert np.allclose(T.T(T.Tt(c)), c, atol=1e-12)
    wc = T.T(np.full((S, N1, N2), 0.7))[0]
    ref = np.zeros_like(wc)
    ref[0, :N1 // 8, :N2 // 8] = math.sqrt(S) * 0.7 * 8.0
    assert np.allclose(wc, ref, atol=1e-10)    # the tabulated taps' zero moment is ~2e-12
    # the same transform as a product of dense per-level operators on one
    # slice: level l applies W_R (x) W_C to the top-left R x C corner only
    # (Mallat's pyramid), W the explicit analysis matrices of the 1D level
    def w1(N):
        g = priors.qmf_highpass(priors.SYM8)
        W = np.zeros((N, N))
        for k in range(N // 2):
            for t in range(16):
                W[k, (2 * k + t) % N] += priors.SYM8[t]
                W[N // 2 + k, (2 * k + t) % N] += g[t]
        return W
    op = np.eye(N1 * N2)
    R, C = N1, N2
    for _ in range(3):
        M = np.eye(N1 * N2)
        idx = (np.arange(R)[:, None] * N2 + np.arange(C)[None, :]).ravel()
        M[np.ix_(idx, idx)] = np.kron(w1(R), w1(C))
        op = M @ op
        R, C = R // 2, C // 2
    per_slice = np.stack([(op @ x[s].ravel()).reshape(N1, N2) for s in range(S)])
    ref = np.tensordot(priors.dct_matrix(S), per_slice, axes=(1, 0))
    assert np.allclose(w[0], ref, atol=1e-12)


def test_wavelet_dct_identity_blur_closed_form():
    """With H = I the wavelet (x) DCT l1 problem is orthonormal-basis
    denoising: ADMM reaches T^T soft(T y, lambda / beta), in both tiers."""
    S, N = 2, 16
    psf = np.zeros((S, S, N, N))
    for s in range(S):
        psf[s, s, 0, 0] = 1.0
    y = _rng(124).standard_normal((S, N, N))
    lam, beta, rho = 0.3, 1.0, 0.7
    T = priors.WaveletDCT(S, N, N, levels=2)
    ref = T.Tt(priors.soft(T.T(y), lam / beta))
    for tier in ("freq", "dense"):
        x, _, _ = admm.AnalysisADMM(psf, "wdct3d", lam, rho, beta, tier=tier,
                                    levels=2).run(y, 400)
        assert np.allclose(x, ref, atol=1e-9)


def test_wavelet_dct_admm_kkt():
    """Algorithm 1 with the wavelet (x) DCT prior reaches a KKT point of
    beta/2 ||y - Hx||^2 + lambda ||T x||_1: beta H^T (Hx - y) + T^T s = 0 with
    s in lambda d||t||_1 at t = T x."""
    x0, psf = _small_problem(K=3, S=3, N1=16, N2=16, seed=45)
    y = model.forward(x0, psf) + 0.01 * _rng(125).standard_normal((3, 16, 16))
    lam, rho, beta = 1e-2, 0.2, 1.0
    alg = admm.AnalysisADMM(psf, "wdct3d", lam, rho, beta, tier="freq", levels=2)
    x, t, u = alg.run(y, 3000)
    w = alg.T.T(x)
    assert np.linalg.norm(w - t) < 1e-7 * np.linalg.norm(w)
    s = rho * u                                   # the scaled dual: s = rho u
    assert np.max(np.abs(s)) <= lam * (1 + 1e-6)
    on = np.abs(t) > 1e-9
    assert np.allclose(s[on], lam * np.sign(t[on]), atol=1e-6 * lam)
    g = beta * model.adjoint(model.forward(x, psf) - y, psf) + alg.T.Tt(s)
    assert np.max(np.abs(g)) < 1e-6 * np.max(np.abs(beta * model.adjoint(y, psf)))


def test_div_is_negative_adjoint_of_grad():
    x = _rng(90).standard_normal((2, 6, 5))
    p = _rng(91).standard_normal((2, 2, 6, 5))
    assert np.isclose(np.vdot(priors.grad2(x), p), -np.vdot(x, priors.div2(p)), rtol=1e-12)


def test_chambolle_meets_the_tv_prox_optimality_conditions():
    """At convergence t = f - mu div p with |p| <= 1 everywhere and
    p . grad t = -|grad t| where grad t != 0: exactly the optimality
    conditions of argmin 1/2 ||t - f||^2 + mu TV_iso(t) (checked directly,
    independently of the iteration's formula). Also TV(t) < TV(f)."""
    f = _rng(92).standard_normal((2, 8, 8))
    mu = 0.3
    t, p = priors.chambolle(f, mu, np.zeros((2, 2, 8, 8)), 20000)
    assert np.allclose(t, f - mu * priors.div2(p), atol=1e-14)
    g = priors.grad2(t)
    ng = np.sqrt(g[0] ** 2 + g[1] ** 2)
    assert np.max(np.sqrt(p[0] ** 2 + p[1] ** 2)) <= 1.0 + 1e-12
    on = ng > 1e-4
    assert np.max(np.abs(p[0] * g[0] + p[1] * g[1] + ng)[on]) < 1e-8
    assert priors.tv_iso(t) < priors.tv_iso(f)
    # the objective is lower than at perturbed points
    obj = lambda z: 0.5 * np.sum((z - f) ** 2) + mu * priors.tv_iso(z)
    for k in range(5):
        assert obj(t) <= obj(t + 1e-3 * _rng(93 + k).standard_normal(t.shape))


def test_chambolle_large_weight_gives_slice_means():
    """With a weight far above the total variation the prox is the constant
    slice mean."""
    f = _rng(98).standard_normal((1, 6, 6))
    t, _ = priors.chambolle(f, 100.0, np.zeros((2, 1, 6, 6)), 20000)
    assert np.allclose(t, f.mean(), atol=1e-6)


def test_itv_admm_with_identity_blur_is_the_tv_prox():
    """With H = I (K = S, delta kernels) the isotropic-TV problem is TV
    denoising of y with weight lambda / beta; ADMM (T = I, Chambolle t-update)
    reaches it."""
    S, N = 2, 8
    psf = np.zeros((S, S, N, N))
    for s in range(S):
        psf[s, s, 0, 0] = 1.0
    y = _rng(99).standard_normal((S, N, N))
    lam, beta, rho = 0.2, 1.0, 0.5
    x, _, _ = admm.AnalysisADMM(psf, "itv2d", lam, rho, beta, tier="freq", inner=50).run(y, 600)
    ref, _ = priors.chambolle(y, lam / beta, np.zeros((2, S, N, N)), 20000)
    assert np.allclose(x, ref, atol=1e-6)
    # isotropic and anisotropic TV give different answers here
    xa = admm.AnalysisADMM(psf, "tv2d", lam, rho, beta, tier="freq").run(y, 600)[0]
    assert np.linalg.norm(xa - x) > 1e-3 * np.linalg.norm(x)


def test_grad3_is_the_explicit_difference_and_div3_its_negative_adjoint():
    """grad3 written out voxel by voxel (circular along the image axes, the
    next slice minus this one along the slices, 0 after the last slice), and
    <grad3 x, p> = -<x, div3 p> for any p (the last slice's band component
    included, which the gradient never fills)."""
    S, N1, N2 = 3, 4, 5
    x = _rng(110).standard_normal((S, N1, N2))
    g = priors.grad3(x)
    for s in range(S):
        for i in range(N1):
            for j in range(N2):
                assert g[0, s, i, j] == x[s, (i + 1) % N1, j] - x[s, i, j]
                assert g[1, s, i, j] == x[s, i, (j + 1) % N2] - x[s, i, j]
                assert g[2, s, i, j] == (x[s + 1, i, j] - x[s, i, j] if s + 1 < S else 0.0)
    p = _rng(111).standard_normal((3, S, N1, N2))
    assert np.isclose(np.vdot(g, p), -np.vdot(x, priors.div3(p)), rtol=1e-12)


def test_div3_grad3_norm_is_below_twelve():
    """The largest eigenvalue of -div3 grad3 on a small cube, from its
    assembled matrix, is 8 + 2 - 2 cos(pi (S - 1) / S) (the circular
    Laplacian's 8 plus the path Laplacian's largest eigenvalue), below 12:
    the step 1/12 meets Chambolle's condition."""
    S, N1, N2 = 3, 4, 4
    n = S * N1 * N2
    A = np.zeros((n, n))
    for k in range(n):
        e = np.zeros(n)
        e[k] = 1.0
        A[:, k] = -priors.div3(priors.grad3(e.reshape(S, N1, N2))).ravel()
    assert np.allclose(A, A.T, atol=1e-12)
    lmax = np.linalg.eigvalsh(A).max()
    assert np.isclose(lmax, 8.0 + 2.0 - 2.0 * np.cos(np.pi * (S - 1) / S), rtol=1e-12)
    assert lmax < 12.0


def test_chambolle3_meets_the_coupled_tv_prox_optimality_conditions():
    """At convergence t = f - mu div3 p with |p| <= 1 and p . grad3 t =
    -|grad3 t| where grad3 t != 0 (the three components' joint norm): the
    optimality conditions of argmin 1/2 ||t - f||^2 + mu TV3(t). The
    objective is lower than at perturbed points."""
    f = _rng(112).standard_normal((3, 6, 6))
    mu = 0.3
    t, p = priors.chambolle3(f, mu, np.zeros((3, 3, 6, 6)), 30000)
    assert np.allclose(t, f - mu * priors.div3(p), atol=1e-14)
    g = priors.grad3(t)
    ng = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
    assert np.max(np.sqrt(p[0] ** 2 + p[1] ** 2 + p[2] ** 2)) <= 1.0 + 1e-12
    on = ng > 1e-3          # a few voxels' gradients are still shrinking to 0 (below 2e-4)
    assert np.max(np.abs(p[0] * g[0] + p[1] * g[1] + p[2] * g[2] + ng)[on]) < 1e-8
    obj = lambda z: 0.5 * np.sum((z - f) ** 2) + mu * priors.tv_iso3(z)
    for k in range(5):
        assert obj(t) <= obj(t + 1e-3 * _rng(113 + k).standard_normal(t.shape))


def test_chambolle3_special_cases():
    """Slices that are all equal have no band variation, so the coupled prox
    is the per-slice prox of one slice, repeated; a single slice is the
    per-slice prox; a weight far above the total variation gives the mean of
    the whole cube (per-slice TV gives each slice's own mean)."""
    f1 = _rng(114).standard_normal((1, 6, 6))
    mu = 0.25
    ref, _ = priors.chambolle(f1, mu, np.zeros((2, 1, 6, 6)), 20000)
    t1, _ = priors.chambolle3(f1, mu, np.zeros((3, 1, 6, 6)), 20000)
    assert np.allclose(t1, ref, atol=1e-9)
    f3 = np.repeat(f1, 3, axis=0)
    t3, _ = priors.chambolle3(f3, mu, np.zeros((3, 3, 6, 6)), 30000)
    assert np.allclose(t3, np.repeat(ref, 3, axis=0), atol=1e-7)
    f = _rng(115).standard_normal((3, 5, 5)) + np.arange(3)[:, None, None]
    tb, _ = priors.chambolle3(f, 100.0, np.zeros((3, 3, 5, 5)), 40000)
    assert np.allclose(tb, f.mean(), atol=1e-5)
    ts, _ = priors.chambolle(f, 100.0, np.zeros((2, 3, 5, 5)), 20000)
    assert np.allclose(ts, f.mean(axis=(1, 2), keepdims=True), atol=1e-6)


def test_itv3_admm_with_identity_blur_is_the_coupled_tv_prox():
    """With H = I the band-coupled isotropic-TV problem is coupled TV
    denoising of y with weight lambda / beta; ADMM (T = I, Chambolle
    t-update along the slices) reaches it, and it differs from the per-slice
    isotropic-TV answer on data that varies along the slices."""
    S, N = 3, 8
    psf = np.zeros((S, S, N, N))
    for s in range(S):
        psf[s, s, 0, 0] = 1.0
    y = _rng(116).standard_normal((S, N, N))
    lam, beta, rho = 0.2, 1.0, 0.5
    x, _, _ = admm.AnalysisADMM(psf, "itv3d", lam, rho, beta, tier="freq", inner=50).run(y, 600)
    ref, _ = priors.chambolle3(y, lam / beta, np.zeros((3, S, N, N)), 30000)
    assert np.allclose(x, ref, atol=1e-6)
    x2 = admm.AnalysisADMM(psf, "itv2d", lam, rho, beta, tier="freq", inner=50).run(y, 600)[0]
    assert np.linalg.norm(x2 - x) > 1e-2 * np.linalg.norm(x)


# ---------------------------------------------------------------- pins added for the larger tiers
@pytest.mark.slow
@pytest.mark.parametrize("N,kind,iters", [(32, "tv2d", 20), (32, "dct2d", 20), (32, "tv3d", 10),
                                          (64, "tv2d", 10)])
def test_dense_and_freq_tiers_agree_at_32_and_64(N, kind, iters):
    """Tier D (assembled normal matrix of Eq. solx_Trans, Cholesky, null-space
    projector for the singular DC block) and tier F (per-frequency solve of
    Eq. solx_Trans_DFT) run the same iteration at 32^2 and 64^2 (K = S = 2,
    S N1 N2 up to 8192 unknowns)."""
    x0, psf = _small_problem(K=2, S=2, N1=N, N2=N, seed=31)
    y = model.forward(x0, psf) + 0.01 * _rng(32).standard_normal((2, N, N))
    lam, rho = (1e-2, 0.1) if kind == "dct2d" else (1e-3, 1e-2)
    a = admm.AnalysisADMM(psf, kind, lam, rho, 1.0, tier="dense").run(y, iters)[0]
    b = admm.AnalysisADMM(psf, kind, lam, rho, 1.0, tier="freq").run(y, iters)[0]
    assert admm.rel_l2(b, a) < 1e-10
    assert np.max(np.abs(b - a)) < 1e-9 * np.max(np.abs(a))


def test_symmlet8_is_the_least_asymmetric_daubechies_factor():
    """The 16-tap filters with 8 vanishing moments are h = sqrt(2) (1 + z^-1)^8
    Q(z) / (norm), with |Q(e^iw)|^2 = P(sin^2(w/2)), P(y) = sum_{k<8}
    C(7+k, k) y^k (Daubechies' construction). Every real spectral factor Q
    picks one zero from each reciprocal pair of P's zeros mapped to z
    (3 complex-conjugate pairs and one real zero: 16 factors). The table
    SYM8 must be the factor whose phase is closest to linear (the
    least-asymmetric choice; measured on Q, the other factor has exactly
    linear phase), and, of that factor and its mirror image (same phase
    nonlinearity), the one whose largest tap is h[7]."""
    import itertools
    c = [math.comb(7 + k, k) for k in range(8)]
    yr = np.roots(c[::-1])
    groups, used = [], set()
    for i, yv in enumerate(yr):
        if i in used:
            continue
        b = 2.0 - 4.0 * yv                       # z + 1/z = 2 - 4 y
        z = (b + np.sqrt(b * b - 4.0 + 0j)) / 2.0
        if abs(yv.imag) < 1e-12:
            groups.append([complex(z)])
            used.add(i)
        else:
            j = [k for k in range(len(yr))
                 if k not in used and k != i and abs(yr[k] - np.conj(yv)) < 1e-8][0]
            used.update([i, j])
            groups.append([z, np.conj(z)])
    assert sorted(len(g) for g in groups) == [1, 2, 2, 2]
    w = np.linspace(0.0, math.pi, 1025)
    A = np.vstack([w, np.ones_like(w)]).T
    found = []
    for choice in itertools.product([0, 1], repeat=len(groups)):
        zs = [(z if ch == 0 else 1.0 / z) for g, ch in zip(groups, choice) for z in g]
        q = np.real(np.poly(zs))
        ph = np.unwrap(np.angle(np.exp(-1j * np.outer(w, np.arange(len(q)))) @ q))
        dev = float(np.max(np.abs(ph - A @ np.linalg.lstsq(A, ph, rcond=None)[0])))
        h = np.convolve(q, [math.comb(8, k) for k in range(9)])
        found.append((dev, h / h.sum() * math.sqrt(2.0)))
    found.sort(key=lambda t: t[0])
    best = [h for d, h in found if d < found[0][0] + 1e-9]
    assert len(best) == 2                         # the factor and its mirror image
    assert found[2][0] > found[0][0] + 0.03       # a clear margin to the next pair
    assert any(np.max(np.abs(h - priors.SYM8)) < 1e-10 for h in best)
    assert int(np.argmax(priors.SYM8)) == 7


# ---------------------------------------------------------------- adaptive penalty, Algorithm 2
def _synth_algs(seed, learn=False, sigma=1.0):
    """A small patch problem and a small 2D convolutional-dictionary problem."""
    S, N = 2, 8
    x0, psf = _small_problem(K=2, S=S, N1=N, N2=N, seed=seed)
    y = model.forward(x0, psf) + 0.01 * _rng(seed + 100).standard_normal((2, N, N))
    D = synth.random_unit_atoms(_rng(seed + 1), 4 * 4 * S, 40)
    filt = synth.random_unit_filters(_rng(seed + 2), 4, 3)

    def patch(rho):
        return admm.PatchADMM(psf, D, 4, 2, 1e-3, rho, 10.0, tier="freq", dict_update=learn,
                              sigma=sigma)

    def conv(rho):
        return admm.ConvADMM(psf, filt, 1e-3, rho, 8.0, tier="freq", dict_update=learn,
                             sigma=sigma)
    return y, patch, conv


@pytest.mark.parametrize("learn", [False, True])
def test_synthesis_adaptive_without_changes_equals_run(learn):
    """With the balance factor so large that neither rho nor sigma changes
    and no stopping, the adaptive run is Algorithm 2 (with its dictionary
    steps) at fixed penalties."""
    y, patch, conv = _synth_algs(50, learn=learn)
    for make in (patch, conv):
        xa, info = make(0.3).run_adaptive(y, 12, mu=1e30, every=1, tol=0.0, adapt_sigma=True)
        xr = make(0.3).run(y, 12)[0]
        assert info["iters"] == 12 and info["rhos"] == [0.3] * 12
        if learn:
            assert info["sigmas"] == [1.0] * 12
        assert np.array_equal(xa, xr)


def test_synthesis_rescaling_keeps_the_fixed_point():
    """Near a fixed point of Algorithm 2 with penalty rho, switching to rho'
    with the scaled dual rescaled by rho / rho' keeps the iterate within the
    drift of two more iterations at rho (rho' u' = rho u leaves the code and
    threshold updates at their fixed point); the opposite rescaling moves it
    ten (conv) to fifty (patch) times further (patch and convolutional
    dictionaries). Two
    iterations: the next x depends on the codes only, the dual acts through
    the code update after it."""
    y, patch, conv = _synth_algs(51)
    rho, rho2 = 0.3, 0.6
    for make in (patch, conv):
        x, z, t, u = make(rho).run(y, 4000)
        drift = np.linalg.norm(make(rho).run(y, 2, state=(z, t, u))[0] - x)
        nxt = make(rho2)
        x_ok = nxt.run(y, 2, state=(z, t, u * rho / rho2))[0]
        x_bad = nxt.run(y, 2, state=(z, t, u * rho2 / rho))[0]
        assert np.linalg.norm(x_ok - x) < 2.0 * drift
        assert np.linalg.norm(x_bad - x) > 5.0 * drift


def test_synthesis_adaptive_moves_rho_and_stops():
    """From a poor penalty in either direction the adaptive run changes rho
    the right way first (up from a tiny rho, where the primal residual
    dominates; down from a huge one), and with the paper's tolerance it stops
    at the first check whose relative change is below it: one check earlier
    the change was still above. (The codes of the synthesis problem are not
    unique, so the limit itself is not pinned here.)"""
    y, patch, conv = _synth_algs(52)
    for make in (patch, conv):
        for rho0, first in ((1e-4, 2.0), (1e3, 0.5)):
            alg = make(rho0)
            x, info = alg.run_adaptive(y, 5000, every=1, tol=1e-4)
            changes = [b / a for a, b in zip(info["rhos"], info["rhos"][1:]) if b != a]
            assert changes and changes[0] == first
            assert info["iters"] < 5000 and info["rel_change"] < 1e-4
            assert alg.rho == rho0
            _, info2 = make(rho0).run_adaptive(y, info["iters"], every=1, tol=0.0)
            assert info2["rel_change"] >= 1e-4      # its last check is at iters - 1


def _split_residuals(alg, y, iters):
    """Run a learning solve; per iteration the change of the scaled dual,
    which is the split residual d - g of that step (e_new - e_old)."""
    es = []
    alg.run(y, iters, callback=lambda *a: es.append(np.array(alg.e, copy=True)))
    res = [np.linalg.norm(es[0])] + [np.linalg.norm(es[k] - es[k - 1]) for k in range(1, iters)]
    return res, max(np.max(np.abs(e)) for e in es)


@pytest.mark.parametrize("dims", [2, 3])
def test_conv_dictionary_admm_converges(dims):
    """Eqs. d_admm, g_admm, h_admm minimise sigma/2 ||d - g + e||^2 over d and
    g, so e is the scaled dual of the split d = g and moves by d - g: the
    split residual then vanishes and e stays bounded. (With the opposite
    sign e doubles every step wherever d follows g - e, and the residual
    grows without bound; here it falls about 300-fold in 60 steps.)"""
    N, M, L = 16, 3, 3
    x0, psf = _small_problem(K=2, S=2, N1=N, N2=N, seed=93)
    y = model.forward(x0, psf) + 0.01 * _rng(94).standard_normal((2, N, N))
    if dims == 2:
        filt = synth.random_unit_filters(_rng(95), M, L)
    else:
        filt = synth.random_unit_filters_3d(_rng(95), M, 2, L)
    alg = admm.ConvADMM(psf, filt, 1e-3, 1.0, 8.0, tier="freq", dims=dims, dict_update=True,
                        sigma=10.0)
    res, emax = _split_residuals(alg, y, 60)
    assert emax < 1.0
    assert res[-1] < 0.05 * res[0]


def test_patch_dictionary_admm_converges():
    """Eqs. ADMM0, ADMM1, subh: the same split as for the convolutional
    dictionary (E the scaled dual of D = G): ||D - G|| vanishes, E stays
    bounded."""
    x0, psf, alg = _patch_dl(96, sigma=0.7)
    y = model.forward(x0, psf) + 0.01 * _rng(97).standard_normal((2, 8, 8))
    res, emax = _split_residuals(alg, y, 60)
    assert emax < 1.0
    assert res[-1] < 0.05 * res[0]
