"""Image-update (x-update) solvers of Section IV.

Analysis case, Eq. solx_Trans:
    x = (rho T^H T + beta H^H H)^(-1) (beta H^H y + rho T^H (t - u))
Synthesis case, Eq. solx_synt:
    x = (c_P I + beta H^H H)^(-1) (beta H^H y + P^H D~ z),   P^H P = c_P I.

Two independent realisations:

* dense tier (tiny grids): the normal matrix is assembled explicitly from the
  dense H of Eq. forwardModel and the dense T^T T, then factorised by Cholesky;
* frequency tier: the DFT diagonalisation of Eq. solx_Trans_DFT /
  solx_synt_DFT, i.e. an S x S Hermitian system at every 2D frequency,
      Psi(w) = rho tau(w) I (+ rho L_band) + beta Lambda(w)^H Lambda(w),
  with Lambda_{k,s}(w) the (unnormalised) DFT of h_{k,s} and tau(w) the DFT
  symbol of T^T T (1 for a unitary T, the circular Laplacian for TV).

Singular normal matrices. With TV on every slice and unit-sum kernels, the DC
block Psi(0) = beta G^T G (G_{k,s} = sum of h_{k,s}) has rank 1, so the
minimiser is not unique (any split of the DC level among bands with the same
blurred sum). The reading used throughout is the minimum-norm minimiser: a
pseudo-inverse that drops eigenvalues below RCOND times the largest one at
that frequency. The dense tier reproduces it with an explicit projector on the
null space (see ``dense_solve``).

Eq. recinv (recursive 2 x 2 block inversion of Psi) is implemented in
``recursive_block_inverse`` and checked against a direct inverse in the tests.

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import solve_triangular

from .model import dense_H

RCOND = 1e-12


# ---------------------------------------------------------------- spectra
def psf_spectra(psf: np.ndarray) -> np.ndarray:
    """Lambda_{k,s}(w): unnormalised 2D DFT of each kernel, shape (K, S, N1, N2).

    With this normalisation DFT(h * x) = Lambda . DFT(x) (convolution theorem)."""
    return np.fft.fft2(psf, axes=(-2, -1))


def gram_blocks(lam: np.ndarray, beta: float, diag_symbol, rho: float,
                band_lap: np.ndarray | None = None) -> np.ndarray:
    """Psi(w) per frequency, shape (N1, N2, S, S) complex.

    Psi_{i,j}(w) = rho * diag_symbol(w) * delta_ij (+ rho * L_band[i, j])
                   + beta * sum_k conj(Lambda_{k,i}(w)) Lambda_{k,j}(w)
    (the block formula below Eq. solx_Trans_DFT, with the identity weighted by
    rho, or by c_P in the synthesis case)."""
    K, S, N1, N2 = lam.shape
    L = np.moveaxis(lam, (0, 1), (2, 3))            # (N1, N2, K, S)
    psi = beta * np.einsum("abki,abkj->abij", np.conj(L), L)
    eye = np.eye(S)[None, None]
    psi = psi + rho * np.asarray(diag_symbol)[..., None, None] * eye
    if band_lap is not None:
        psi = psi + rho * band_lap[None, None]
    return psi


def hermitian_pinv(psi: np.ndarray, rcond: float = RCOND) -> np.ndarray:
    """Batched pseudo-inverse of Hermitian S x S blocks by eigendecomposition;
    eigenvalues <= rcond * max eigenvalue (per block) are treated as zero."""
    w, V = np.linalg.eigh(psi)
    wmax = np.max(np.abs(w), axis=-1, keepdims=True)
    keep = w > rcond * wmax
    inv = np.where(keep, 1.0 / np.where(keep, w, 1.0), 0.0)
    return np.einsum("...ik,...k,...jk->...ij", V, inv, np.conj(V))


def recursive_block_inverse(psi: np.ndarray) -> np.ndarray:
    """Eq. recinv applied recursively: split Psi into [[P11, P12], [P21, P22]],
        B = -(P22 - P21 P11^-1 P12)^-1,
        A = P11^-1 - P11^-1 P12 B P21 P11^-1,
        Psi^-1 = [[A, P11^-1 P12 B], [B P21 P11^-1, -B]],
    recursing on P11 and on the Schur complement. Works on batches (..., S, S);
    every block of the paper's Psi is diagonal in frequency, so this is the
    same computation done independently at each frequency. Nonsingular only."""
    S = psi.shape[-1]
    if S == 1:
        return 1.0 / psi
    h = (S + 1) // 2
    P11, P12 = psi[..., :h, :h], psi[..., :h, h:]
    P21, P22 = psi[..., h:, :h], psi[..., h:, h:]
    P11i = recursive_block_inverse(P11)
    B = -recursive_block_inverse(P22 - P21 @ P11i @ P12)
    A = P11i - P11i @ P12 @ B @ P21 @ P11i
    top = np.concatenate([A, P11i @ P12 @ B], axis=-1)
    bot = np.concatenate([B @ P21 @ P11i, -B], axis=-1)
    return np.concatenate([top, bot], axis=-2)


# ---------------------------------------------------------------- frequency tier
class FreqSolver:
    """Per-frequency x-update (Eq. solx_Trans_DFT / solx_synt_DFT) in FP64.

    ``weight`` is rho for the analysis case (identity weighted by rho times the
    symbol of T^T T) or c_P for the synthesis case (symbol 1)."""

    def __init__(self, psf, beta, weight, diag_symbol, band_lap=None, rcond=RCOND):
        self.lam = psf_spectra(psf)
        self.beta = float(beta)
        self.psi = gram_blocks(self.lam, beta, diag_symbol, weight, band_lap)
        self.psi_pinv = hermitian_pinv(self.psi, rcond)

    def data_term(self, y):
        """beta Lambda^H (F y), shape (S, N1, N2) complex (Alg. 1/2, step 2)."""
        yh = np.fft.fft2(y, axes=(-2, -1))
        return self.beta * np.einsum("ksab,kab->sab", np.conj(self.lam), yh)

    def solve_hat(self, rhs_hat):
        """x_hat(w) = Psi(w)^+ rhs_hat(w) at every frequency."""
        return np.einsum("abij,jab->iab", self.psi_pinv, rhs_hat)

    def solve(self, bhat, extra_spatial):
        """x = F^-1 Psi^+ (bhat + F extra_spatial); ``extra_spatial`` is
        rho T^H (t - u) (analysis) or P^H D~ z (synthesis)."""
        rhs = bhat + np.fft.fft2(extra_spatial, axes=(-2, -1))
        return np.ascontiguousarray(np.real(np.fft.ifft2(self.solve_hat(rhs), axes=(-2, -1))))


# ---------------------------------------------------------------- dense tier
def dense_TtT(transform, S, N1, N2) -> np.ndarray:
    """Dense T^T T, assembled by applying T^T T to every unit vector."""
    n = S * N1 * N2
    out = np.empty((n, n))
    e = np.zeros((S, N1, N2))
    for i in range(n):
        e.flat[i] = 1.0
        out[:, i] = transform.Tt(transform.T(e)).ravel()
        e.flat[i] = 0.0
    return out


class DenseSolver:
    """x-update by a dense Cholesky solve of the normal equations
    (Eq. solx_Trans / solx_synt), for grids with S N1 N2 <= 8192.

    ``reg`` is the dense regulariser matrix: rho T^T T (analysis) or c_P I
    (synthesis). If T annihilates per-band constants (TV on slices), the DC
    null space of the normal matrix is {x_s = c_s 1 : G c = 0}; its projector
    P_N = (N_c N_c^T) (x) (1 1^T / N1 N2) is added before factorising and the
    solution is projected off it, which yields the minimum-norm minimiser."""

    def __init__(self, psf, beta, reg, annihilates_constants=False, rcond=RCOND):
        K, S, N1, N2 = psf.shape
        self.S, self.N1, self.N2 = S, N1, N2
        H = dense_H(psf)
        self.H = H
        self.beta = float(beta)
        A = beta * (H.T @ H) + reg
        self.PN = None
        if annihilates_constants:
            G = psf.sum(axis=(2, 3))                  # (K, S)
            w, V = np.linalg.eigh(beta * G.T @ G)
            null = V[:, w <= rcond * np.max(np.abs(w))]
            if null.shape[1]:
                ones = np.ones(N1 * N2) / np.sqrt(N1 * N2)
                Nb = np.kron(null, ones[:, None])     # (S N1 N2, dim null)
                self.PN = Nb @ Nb.T
                A = A + self.PN
        self.L = np.linalg.cholesky(A)

    def solve(self, rhs_spatial):
        """x = A^+ rhs for a spatial right-hand side of shape (S, N1, N2)."""
        r = rhs_spatial.ravel()
        if self.PN is not None:
            r = r - self.PN @ r
        # L L^T x = r by forward then backward substitution
        z = solve_triangular(self.L, r, lower=True)
        x = solve_triangular(self.L.T, z, lower=False)
        if self.PN is not None:
            x = x - self.PN @ x
        return x.reshape(self.S, self.N1, self.N2)

    def data_term(self, y):
        """beta H^T y (spatial)."""
        return (self.beta * (self.H.T @ y.ravel())).reshape(self.S, self.N1, self.N2)
