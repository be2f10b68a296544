"""Algorithms 1 and 2 of Section IV, step by step, in FP64.

Algorithm 1 (analysis case; Eqs. analysis_ADMM, iter_ADMM1, iter_ADMM2,
subu_trans), with t^0 = u^0 = 0 (the paper leaves them to choice):
    x^{l+1} = (rho T^H T + beta H^H H)^+ (beta H^H y + rho T^H (t^l - u^l))
    t^{l+1} = soft(T x^{l+1} + u^l, lambda / rho)
    u^{l+1} = u^l + T x^{l+1} - t^{l+1}

Algorithm 2 (synthesis case; Eqs. synthesis_ADMM, iterd_ADMM1..3, subu_dic),
with z^0 = t^0 = u^0 = 0:
    x^{l+1} = (c_P I + beta H^H H)^-1 (beta H^H y + P^H D~ z^l)
    z^{l+1} = argmin_z 1/2 ||D~ z - P x^{l+1}||^2 + rho/2 ||z - t^l + u^l||^2
        patch dictionary:  z_j = (rho I + D^T D)^-1 (D^T P_j x + rho (t_j - u_j))
                           (Eq. solz_patch2)
        conv dictionary:   (rho I + Theta^H Theta) F z = Theta^H F x + rho F (t - u)
                           solved per frequency by Sherman-Morrison
                           (Eqs. solz_DFT, solz_DFT_SM)
    t^{l+1} = soft(z^{l+1} + u^l, lambda / rho)          (Eq. softADMM)
    u^{l+1} = u^l + z^{l+1} - t^{l+1}

The penalty rho is fixed and a fixed number of iterations is run (the paper's
adaptive rho and relative-change stopping rule, Section IV-C, are not part of
this reference). Iterations return x^L.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np

from . import model, priors, xupdate


def _tier(S, N1, N2, tier):
    if tier == "auto":
        return "dense" if S * N1 * N2 <= 2048 else "freq"
    return tier


# ================================================================ analysis
def analysis_objective(x, y, psf, transform, lam, beta):
    """beta/2 ||y - Hx||^2 + lambda ||T x||_1 (Eq. rls with Eq. analysis)."""
    r = y - model.forward(x, psf)
    return 0.5 * beta * np.sum(r * r) + lam * np.sum(np.abs(transform.T(x)))


class AnalysisADMM:
    """Algorithm 1 for T in {dct2d, dct3d, tv2d, tv3d, wdct3d (Symmlet-8
    wavelet per slice, `levels` levels, then DCT along the bands)} and
    Phi = l1, and for
    isotropic TV ("itv2d": T = I, Phi = TV of every slice, t-update by
    Chambolle's algorithm with `inner` iterations per ADMM iteration,
    warm-started from the previous dual p, step 1/8; "itv3d": the same with
    the gradient coupled along the slices, step 1/12)."""

    def __init__(self, psf, kind, lam, rho, beta=1.0, tier="auto", inner=20, levels=3):
        K, S, N1, N2 = psf.shape
        self.psf = psf
        self.kind = kind
        self.K, self.S, self.N1, self.N2 = K, S, N1, N2
        self.lam, self.beta = float(lam), float(beta)
        self.T = priors.make_transform(kind, S, N1, N2, levels)
        self.tier = _tier(S, N1, N2, tier)
        self.inner = int(inner)
        self.set_rho(rho)

    def t_update(self, v, kappa, p):
        """Eq. solt_trans for Phi = l1 (soft threshold of v = Tx + u); for
        isotropic TV the TV proximal map of v by Chambolle's algorithm.
        Returns (t, p) (p: the TV dual, None for l1)."""
        if self.kind == "itv2d":
            if p is None:
                p = np.zeros((2,) + v.shape[1:])
            t, p = priors.chambolle(v[0], kappa, p, self.inner)
            return t[None], p
        if self.kind == "itv3d":
            if p is None:
                p = np.zeros((3,) + v.shape[1:])
            t, p = priors.chambolle3(v[0], kappa, p, self.inner)
            return t[None], p
        return priors.soft(v, kappa), None

    def set_rho(self, rho):
        """(Re)build the x-update for penalty rho (Psi depends on rho)."""
        self.rho = float(rho)
        S, N1, N2 = self.S, self.N1, self.N2
        if self.tier == "dense":
            reg = self.rho * xupdate.dense_TtT(self.T, S, N1, N2)
            self.solver = xupdate.DenseSolver(
                self.psf, self.beta, reg, annihilates_constants=(self.kind == "tv2d"))
        else:
            band_lap = self.T.band_laplacian() if self.kind == "tv3d" else None
            self.solver = xupdate.FreqSolver(
                self.psf, self.beta, self.rho, self.T.gram_symbol(N1, N2), band_lap)

    def x_update(self, data, t, u):
        extra = self.rho * self.T.Tt(t - u)
        if self.tier == "dense":
            return self.solver.solve(data + extra)
        return self.solver.solve(data, extra)

    def run(self, y, iters, callback=None, state=None):
        """Run ``iters`` iterations from t = u = 0 (or from ``state``).
        Returns (x, t, u)."""
        data = self.solver.data_term(y)
        if state is None:
            t = np.zeros(self.T.shape)
            u = np.zeros(self.T.shape)
        else:
            t, u = (a.copy() for a in state)
        x = None
        kappa = self.lam / self.rho
        p = None
        for it in range(iters):
            x = self.x_update(data, t, u)
            w = self.T.T(x)
            t_new, p = self.t_update(w + u, kappa, p)
            u = u + w - t_new
            t = t_new
            if callback is not None:
                callback(it, x, t, u)
        return x, t, u

    def run_adaptive(self, y, max_iters, tau=2.0, mu=10.0, every=1, tol=1e-4):
        """Algorithm 1 with the penalty update and stopping rule of Section
        IV-C (Eq. paramS). At every `every`-th iteration l < max_iters (the
        paper does not say when to check; the last iterate is returned
        either way), after the t- and u-updates:
          r = ||T x^l - t^l||,  s = rho ||t^l - t^{l-1}||;
          stop (returning x^l) if ||x^l - x^{l-1}|| / ||x^{l-1}|| < tol;
          rho <- tau rho if r > mu s, rho / tau if s > mu r;
          on a change the scaled dual is rescaled, u <- u rho_old / rho_new,
          and the x-update is rebuilt for the new rho.
        Returns (x, info) with info = dict(iters, rho, rhos, rel_change, r, s)."""
        rho0 = self.rho
        data = self.solver.data_term(y)
        t = np.zeros(self.T.shape)
        u = np.zeros(self.T.shape)
        x_prev = None
        rhos = [self.rho]
        info = {"rel_change": None, "r": None, "s": None}
        it = 0
        x = None
        p = None
        for it in range(1, max_iters + 1):
            x = self.x_update(data, t, u)
            w = self.T.T(x)
            kappa = self.lam / self.rho
            t_new, p = self.t_update(w + u, kappa, p)
            u_new = u + w - t_new
            if it % every == 0 and it < max_iters:   # the last iterate is returned anyway
                r = float(np.linalg.norm(w - t_new))
                s_ = self.rho * float(np.linalg.norm(t_new - t))
                info["r"], info["s"] = r, s_
                if x_prev is not None:
                    rel = float(np.linalg.norm(x - x_prev) / np.linalg.norm(x_prev))
                    info["rel_change"] = rel
                    if rel < tol:
                        break
                new = self.rho
                if r > mu * s_:
                    new = tau * self.rho
                elif s_ > mu * r:
                    new = self.rho / tau
                if new != self.rho:
                    u_new = u_new * (self.rho / new)
                    self.set_rho(new)
                    data = self.solver.data_term(y)
                rhos.append(self.rho)
            t, u = t_new, u_new
            x_prev = x
        info.update(iters=it, rho=self.rho, rhos=rhos)
        self.set_rho(rho0)
        return x, info

    def kkt(self, y, x, t, u):
        """Relative KKT residuals of the split problem at (x, t, u):
        primal ||Tx - t||, stationarity in x ||beta H^T (Hx - y) + rho T^T u||,
        and the prox fixed point ||t - soft(t + u, lambda/rho)||."""
        Tx = self.T.T(x)
        r1 = np.linalg.norm(Tx - t) / max(np.linalg.norm(Tx), 1e-300)
        g = self.beta * model.adjoint(model.forward(x, self.psf) - y, self.psf) \
            + self.rho * self.T.Tt(u)
        r2 = np.linalg.norm(g) / max(
            np.linalg.norm(self.beta * model.adjoint(y, self.psf)), 1e-300)
        r3 = np.linalg.norm(t - priors.soft(t + u, self.lam / self.rho)) / max(
            np.linalg.norm(t), 1e-300)
        return r1, r2, r3


# ================================================================ synthesis: patches
class PatchADMM:
    """Algorithm 2 with the patch-based dictionary prior.

    D has shape (n, A) with n = Q*Q*S (column a = atom a, element layout as in
    ``priors.Patches``); codes z, t, u have shape (A, J).

    dict_update: learn the dictionary online (Section IV-B, patch-based
    dictionary update): after the code update of each outer iteration one
    step of the dictionary ADMM, Eqs. ADMM0 (closed form Eq. sold_patch),
    ADMM1 (projection onto ||G||_F = 1, the constraint of Eq.
    patch_based_dic) and subh, starting from G = D, E = 0; the next x- and
    z-updates use G."""

    def __init__(self, psf, D, Q, stride, lam, rho, beta, tier="auto", dict_update=False,
                 sigma=1.0):
        K, S, N1, N2 = psf.shape
        self.psf = psf
        self.S, self.N1, self.N2 = S, N1, N2
        self.D = np.asarray(D, dtype=np.float64)
        self.P = priors.Patches(S, N1, N2, Q, stride)
        assert self.D.shape[0] == self.P.n
        self.lam, self.rho, self.beta = float(lam), float(rho), float(beta)
        self.tier = _tier(S, N1, N2, tier)
        cP = self.P.c_P
        if self.tier == "dense":
            self.solver = xupdate.DenseSolver(psf, beta, cP * np.eye(S * N1 * N2))
        else:
            self.solver = xupdate.FreqSolver(psf, beta, cP, np.ones((N1, N2)))
        self.dict_update, self.sigma = bool(dict_update), float(sigma)
        self.g = self.D.copy()
        self.e = np.zeros_like(self.D)
        self.set_dictionary(self.D)

    def set_dictionary(self, D):
        """Use dictionary D in the following x- and z-updates."""
        self.D = np.array(D, dtype=np.float64)
        A = self.D.shape[1]
        self.zgram = self.rho * np.eye(A) + self.D.T @ self.D     # rho I + D^T D

    def set_rho(self, rho):
        """Penalty rho of the code split (the z-update matrix depends on it)."""
        self.rho = float(rho)
        self.set_dictionary(self.D)

    def run_adaptive(self, y, max_iters, tau=2.0, mu=10.0, every=1, tol=1e-4,
                     adapt_sigma=False):
        """Algorithm 2 with the penalty update and stopping rule of Section
        IV-C; see ``synthesis_run_adaptive``."""
        return synthesis_run_adaptive(self, y, max_iters, tau, mu, every, tol, adapt_sigma)

    def d_update_patches(self, X, z):
        """Eq. sold_patch: D = (X Z^T + sigma (G - E)) (Z Z^T + sigma I)^-1
        for patch matrix X (n x J) and codes Z (A x J); the system matrix
        is symmetric, so D^T solves (Z Z^T + sigma I) D^T = (X Z^T +
        sigma (G - E))^T."""
        A = z.shape[0]
        rhs = X @ z.T + self.sigma * (self.g - self.e)
        return np.linalg.solve(z @ z.T + self.sigma * np.eye(A), rhs.T).T

    def d_update(self, x, z):
        """Eq. ADMM0 with X = [P_1 x | ... | P_J x]."""
        return self.d_update_patches(self.P.extract(x), z)

    def g_update(self, d):
        """Eq. ADMM1: the point of the unit Frobenius sphere nearest to
        D + E, i.e. (D + E) / ||D + E||_F."""
        w = d + self.e
        return w / np.linalg.norm(w)

    def x_update(self, data, z):
        extra = self.P.adjoint(self.D @ z)                    # P^H D~ z
        if self.tier == "dense":
            return self.solver.solve(data + extra)
        return self.solver.solve(data, extra)

    def z_update(self, x, t, u):
        """Eq. solz_patch2 for all patches at once."""
        rhs = self.D.T @ self.P.extract(x) + self.rho * (t - u)
        return np.linalg.solve(self.zgram, rhs)

    def run(self, y, iters, callback=None, state=None):
        """Run ``iters`` iterations from z = t = u = 0 (or from ``state`` =
        (z, t, u)). Returns (x, z, t, u)."""
        data = self.solver.data_term(y)
        A = self.D.shape[1]
        z = np.zeros((A, self.P.J))
        t = np.zeros_like(z)
        u = np.zeros_like(z)
        if state is not None:
            z, t, u = (np.array(a, dtype=np.float64) for a in state)
        kappa = self.lam / self.rho
        x = None
        for it in range(iters):
            x = self.x_update(data, z)
            z = self.z_update(x, t, u)
            t_new = priors.soft(z + u, kappa)
            u = u + z - t_new
            t = t_new
            if self.dict_update:
                # one D, G, E step per outer iteration (Eqs. ADMM0, ADMM1,
                # subh); the next x- and z-updates use the feasible G. The
                # scaled dual of the penalty sigma/2 ||D - G + E||^2 that
                # ADMM0 and ADMM1 minimise moves by the split residual D - G
                # (the sign printed with Eq. subh, G - D, makes E double
                # every step where D follows G - E, and the solve diverge)
                d = self.d_update(x, z)
                g = self.g_update(d)
                self.e = self.e + d - g
                self.g = g
                self.set_dictionary(g)
            if callback is not None:
                callback(it, x, z, t, u)
        return x, z, t, u


# ================================================================ synthesis: conv dictionary
def sherman_morrison(theta, c, rho):
    """Eq. solz_DFT_SM at every frequency: solve (rho I + a a^H) v = c for the
    M-vector v, where a = conj(theta) collects the filter spectra at that
    frequency (so that Theta^H Theta = a a^H):
        v = rho^-1 (c - a (a^H c) / (rho + a^H a)).
    theta: (M, ...) complex; c: (M, ...) complex; rho: scalar, or an array
    broadcasting over the frequency axes (a diagonal that varies with the
    frequency, as with the Tikhonov term)."""
    a = np.conj(theta)
    ahc = np.sum(np.conj(a) * c, axis=0)
    aha = np.sum(np.abs(a) ** 2, axis=0)
    return (c - a * (ahc / (rho + aha))[None]) / rho


class ConvADMM:
    """Algorithm 2 with a common 2D convolutional dictionary for every band
    (P = I, c_P = 1), or with 3D filters and codes (dims=3). Codes z, t, u
    have shape (M, S, N1, N2). mu > 0 adds
    the gradient (Tikhonov) term of Eq. DL_PriorHP_conv; the z-update normal
    equation then gains mu sum_i R_i^H R_i on its left-hand side (stated
    below Eq. solz), diagonal in frequency with symbol psi(w)."""

    def __init__(self, psf, filters, lam, rho, beta, tier="auto", mu=0.0, dims=2,
                 dict_update=False, sigma=10.0):
        K, S, N1, N2 = psf.shape
        self.psf = psf
        self.S, self.N1, self.N2 = S, N1, N2
        self.dims = int(dims)
        if self.dims == 3:
            # 3D filters (M, S, L, L) and codes: every operator is diagonal
            # in the 3D DFT over (band, n1, n2)
            assert mu == 0.0, "the gradient term is defined here for 2D codes only"
            self.cd = priors.ConvDict3D(np.asarray(filters, dtype=np.float64), S, N1, N2)
        else:
            self.cd = priors.ConvDict2D(np.asarray(filters, dtype=np.float64), S, N1, N2)
        self.M = self.cd.M
        self.lam, self.rho, self.beta = float(lam), float(rho), float(beta)
        self.tier = _tier(S, N1, N2, tier)
        if self.tier == "dense":
            self.solver = xupdate.DenseSolver(psf, beta, np.eye(S * N1 * N2))
        else:
            self.solver = xupdate.FreqSolver(psf, beta, 1.0, np.ones((N1, N2)))
        self.theta = self.cd.spectra()                           # (M, N1, N2)
        self.dict_update = bool(dict_update)
        if self.dict_update:
            # online dictionary update (Eqs. d_admm, g_admm, h_admm)
            L = np.asarray(filters).shape[-1]
            self.sigma = float(sigma)
            self.support = priors.filter_on_grid(np.ones((L, L)), N1, N2) > 0   # (N1, N2)
            self.g = self.cd.h.copy()                            # feasible dictionary
            self.e = np.zeros_like(self.g)                       # scaled dual
        self.mu = float(mu)
        self.psi = priors.tikhonov_symbol(N1, N2)                # (N1, N2)

    def synth(self, z):
        if self.tier == "dense":
            return self.cd.synth(z)
        if self.dims == 3:
            zh = np.fft.fftn(z, axes=(1, 2, 3))
            return np.ascontiguousarray(np.real(np.fft.ifftn(
                np.einsum("msab,msab->sab", self.theta, zh), axes=(0, 1, 2))))
        zh = np.fft.fft2(z, axes=(-2, -1))
        return np.ascontiguousarray(np.real(np.fft.ifft2(
            np.einsum("mab,msab->sab", self.theta, zh), axes=(-2, -1))))

    def x_update(self, data, z):
        extra = self.synth(z)
        if self.tier == "dense":
            return self.solver.solve(data + extra)
        return self.solver.solve(data, extra)

    def z_update(self, x, t, u):
        """Eq. solz_DFT: c = Theta^H F x + rho F (t - u), then Sherman-Morrison
        per frequency and per band (diagonal rho + mu psi(w)), then inverse
        DFT."""
        if self.dims == 3:
            # the same Sherman-Morrison solve at every 3D frequency
            xh = np.fft.fftn(x, axes=(0, 1, 2))                  # (S, N1, N2)
            gh = np.fft.fftn(t - u, axes=(1, 2, 3))              # (M, S, N1, N2)
            c = np.conj(self.theta) * xh[None] + self.rho * gh
            v = sherman_morrison(self.theta, c, self.rho)
            return np.ascontiguousarray(np.real(np.fft.ifftn(v, axes=(1, 2, 3))))
        xh = np.fft.fft2(x, axes=(-2, -1))                       # (S, N1, N2)
        gh = np.fft.fft2(t - u, axes=(-2, -1))                   # (M, S, N1, N2)
        c = np.conj(self.theta)[:, None] * xh[None] + self.rho * gh
        v = sherman_morrison(self.theta[:, None], c, self.rho + self.mu * self.psi)
        return np.ascontiguousarray(np.real(np.fft.ifft2(v, axes=(-2, -1))))

    def d_update(self, x, z):
        """Eq. sold_3D: (sigma I + Z^H Z) d = Z^H x + sigma (g - e), Z_m the
        3D convolution by code z_m, diagonal in the 3D DFT (rank one per
        frequency plus sigma I): Sherman-Morrison at every 3D frequency.
        d is full size (M, S, N1, N2). 2D form (common filters, the sum over
        the planes of Section IV-B's remark): per 2D frequency the M x M
        system sigma I + sum_s conj(Z_s) Z_s^T (rank S plus sigma I), solved
        directly; d has shape (M, N1, N2)."""
        if self.dims == 2:
            xh = np.fft.fft2(x, axes=(-2, -1))                   # (S, N1, N2)
            zh = np.fft.fft2(z, axes=(-2, -1))                   # (M, S, N1, N2)
            geh = np.fft.fft2(self.g - self.e, axes=(-2, -1))    # (M, N1, N2)
            rhs = np.einsum("msab,sab->mab", np.conj(zh), xh) + self.sigma * geh
            mat = np.einsum("msab,nsab->abmn", np.conj(zh), zh)
            mat = mat + self.sigma * np.eye(self.M)[None, None]
            dh = np.linalg.solve(mat, np.moveaxis(rhs, 0, -1)[..., None])[..., 0]
            return np.ascontiguousarray(np.real(np.fft.ifft2(np.moveaxis(dh, -1, 0),
                                                             axes=(-2, -1))))
        xh = np.fft.fftn(x, axes=(0, 1, 2))
        zh = np.fft.fftn(z, axes=(1, 2, 3))
        c = np.conj(zh) * xh[None] + self.sigma * np.fft.fftn(self.g - self.e, axes=(1, 2, 3))
        dh = sherman_morrison(zh, c, self.sigma)
        return np.ascontiguousarray(np.real(np.fft.ifftn(dh, axes=(1, 2, 3))))

    def g_update(self, d):
        """Eq. g_admm (with e^l, the readable form of the garbled index):
        crop d + e to the L x L x S filter support and scale every filter to
        unit l2 norm (projection onto the constraint set C_d)."""
        mask = self.support if self.dims == 2 else self.support[None]
        w = (d + self.e) * mask[None]
        n = np.sqrt(np.sum(w.reshape(self.M, -1) ** 2, axis=1))
        return w / n.reshape((self.M,) + (1,) * (w.ndim - 1))

    def set_dictionary(self, g):
        self.cd.h = g
        self.theta = self.cd.spectra()

    def set_rho(self, rho):
        """Penalty rho of the code split (used directly by the z-update)."""
        self.rho = float(rho)

    def run_adaptive(self, y, max_iters, tau=2.0, mu=10.0, every=1, tol=1e-4,
                     adapt_sigma=False):
        """Algorithm 2 with the penalty update and stopping rule of Section
        IV-C; see ``synthesis_run_adaptive``."""
        return synthesis_run_adaptive(self, y, max_iters, tau, mu, every, tol, adapt_sigma)

    def run(self, y, iters, callback=None, state=None):
        """Run ``iters`` iterations from z = t = u = 0 (or from ``state`` =
        (z, t, u)). Returns (x, z, t, u)."""
        data = self.solver.data_term(y)
        z = np.zeros((self.M, self.S, self.N1, self.N2))
        t = np.zeros_like(z)
        u = np.zeros_like(z)
        if state is not None:
            z, t, u = (np.array(a, dtype=np.float64) for a in state)
        kappa = self.lam / self.rho
        x = None
        for it in range(iters):
            x = self.x_update(data, z)
            z = self.z_update(x, t, u)
            t_new = priors.soft(z + u, kappa)
            u = u + z - t_new
            t = t_new
            if self.dict_update:
                # one d, g, e step per outer iteration; the next x- and
                # z-updates use the feasible dictionary g
                d = self.d_update(x, z)
                g = self.g_update(d)
                self.e = self.e + d - g      # Eq. h_admm, sign as for Eq. subh
                self.g = g
                self.set_dictionary(g)
            if callback is not None:
                callback(it, x, z, t, u)
        return x, z, t, u


def synthesis_run_adaptive(alg, y, max_iters, tau=2.0, mu=10.0, every=1, tol=1e-4,
                           adapt_sigma=False):
    """Algorithm 2 (patch or convolutional dictionary) with the penalty update
    and stopping rule of Section IV-C (Eq. paramS). The split is z = t, so at
    every `every`-th iteration l < max_iters, after the t- and u-updates:
      r = ||z^l - t^l||,  s = rho ||t^l - t^{l-1}||;
      stop (returning x^l) if ||x^l - x^{l-1}|| / ||x^{l-1}|| < tol;
      rho <- tau rho if r > mu s, rho / tau if s > mu r; on a change the
      scaled dual is rescaled, u <- u rho_old / rho_new, and the code update
      is rebuilt for the new rho (its threshold lambda / rho too).
    With online dictionary learning and adapt_sigma (the paper applies the
    same strategy to sigma in the dictionary update), after the D, G, E step
    of a checked iteration:
      r_d = ||D - G||,  s_d = sigma ||G - G_prev||;
      sigma <- tau sigma if r_d > mu s_d, sigma / tau if s_d > mu r_d, and
      the scaled dual E is rescaled by sigma_old / sigma_new.
    The object is left with its starting rho and sigma (and dictionary: the
    learned one, as after ``run``). Returns (x, info), info = dict(iters,
    rho, rhos, sigma, sigmas, rel_change, r, s, trace = [(l, r, s, c)] of the
    checks, trace_sigma = [(l, r_d, s_d)] of the sigma checks)."""
    rho0 = alg.rho
    learn = getattr(alg, "dict_update", False)
    sig0 = alg.sigma if learn else None
    data = alg.solver.data_term(y)
    zshape = (alg.D.shape[1], alg.P.J) if hasattr(alg, "P") else \
        (alg.M, alg.S, alg.N1, alg.N2)
    z = np.zeros(zshape)
    t = np.zeros(zshape)
    u = np.zeros(zshape)
    x_prev, x = None, None
    rhos, sigmas = [alg.rho], ([alg.sigma] if learn else [])
    info = {"rel_change": None, "r": None, "s": None, "trace": [], "trace_sigma": []}
    it = 0
    for it in range(1, max_iters + 1):
        x = alg.x_update(data, z)
        z = alg.z_update(x, t, u)
        kappa = alg.lam / alg.rho
        t_new = priors.soft(z + u, kappa)
        u_new = u + z - t_new
        check = it % every == 0 and it < max_iters   # the last iterate is returned anyway
        if check:
            r = float(np.linalg.norm(z - t_new))
            s_ = alg.rho * float(np.linalg.norm(t_new - t))
            info["r"], info["s"] = r, s_
            rel = None
            if x_prev is not None:
                rel = float(np.linalg.norm(x - x_prev) / np.linalg.norm(x_prev))
                info["rel_change"] = rel
            info["trace"].append((it, r, s_, rel))
            if rel is not None and rel < tol:
                break
            new = alg.rho
            if r > mu * s_:
                new = tau * alg.rho
            elif s_ > mu * r:
                new = alg.rho / tau
            if new != alg.rho:
                u_new = u_new * (alg.rho / new)
                alg.set_rho(new)
            rhos.append(alg.rho)
        t, u = t_new, u_new
        if learn:
            g_prev = alg.g
            d = alg.d_update(x, z)
            g = alg.g_update(d)
            alg.e = alg.e + d - g
            alg.g = g
            if check and adapt_sigma:
                rd = float(np.linalg.norm(d - g))
                sd = alg.sigma * float(np.linalg.norm(g - g_prev))
                info["trace_sigma"].append((it, rd, sd))
                new = alg.sigma
                if rd > mu * sd:
                    new = tau * alg.sigma
                elif sd > mu * rd:
                    new = alg.sigma / tau
                if new != alg.sigma:
                    alg.e = alg.e * (alg.sigma / new)
                    alg.sigma = new
                sigmas.append(alg.sigma)
            alg.set_dictionary(g)
        x_prev = x
    info.update(iters=it, rho=alg.rho, rhos=rhos,
                sigma=alg.sigma if learn else None, sigmas=sigmas)
    alg.set_rho(rho0)
    if learn:
        alg.sigma = sig0
    return x, info


def psnr(x, ref, peak=1.0):
    """10 log10(peak^2 / MSE) over all voxels (peak 1 for data in [0, 1])."""
    mse = np.mean((np.asarray(x) - np.asarray(ref)) ** 2)
    return 10.0 * np.log10(peak * peak / mse)


def rel_l2(a, b):
    """||a - b|| / ||b||."""
    return float(np.linalg.norm(np.ravel(a) - np.ravel(b)) / np.linalg.norm(np.ravel(b)))
