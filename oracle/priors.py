"""Priors of Section III and their elementary operators.

* Analysis prior R(x) = lambda * ||T x||_1 (Eq. analysis with Phi = l1):
  - T = orthonormal 2D DCT-II applied to each slice (a unitary transform, so
    T^H T = I as assumed below Eq. solx_Trans), or the same followed by the
    orthonormal DCT-II along the band axis (one 3D transform);
  - T = anisotropic discrete gradient on each slice (circular forward
    differences along both image axes; "multidimensional discrete derivative
    operators" of Section III-A);
  - T = the same plus a forward difference along the band axis (3D case,
    non-circular, no term after the last band);
  - T = 2D Symmlet-8 wavelet transform of each slice followed by the
    orthonormal DCT-II along the band axis (the Kronecker basis used for the
    analysis prior in Section V-A).
* Isotropic TV (Phi = TV with T = I, Section III-A): the Euclidean norm of
  the per-slice gradient, or of the gradient with its band component (the
  same band difference as the 3D anisotropic case), and its proximal map by
  Chambolle's projection algorithm.
* Soft thresholding, the l1 proximal map (Eq. solt_trans), sign(0) = -1.
* Patch extraction P_j for Q x Q x T patches spanning all bands (Eq.
  patch_based), extracted circularly at a fixed stride.
* Convolutional dictionary synthesis for 2D correlations: each band is
  sum_m d_m * z_{m,s} with a common set of L x L filters (the 2D-correlation
  variant of Eq. conv_dic, Section III-B.2), optionally with gradient
  (Tikhonov) regularisation of the codes (Eq. DL_PriorHP_conv, 2D case:
  gradients along the first and second image axes); and with 3D filters and
  codes (circular along the bands too, diagonal in the 3D DFT).

TEST INFRASTRUCTURE ONLY (see the package docstring).
"""
from __future__ import annotations

import math

import numpy as np

from .model import conv_circ, corr_circ


# ---------------------------------------------------------------- soft threshold
def soft(w: np.ndarray, tau: float) -> np.ndarray:
    """Eq. solt_trans: w_i -> sign(w_i) max(|w_i| - tau, 0), sign(w) = 1 if
    w > 0 else -1 (the value at w = 0 is 0 either way)."""
    sgn = np.where(w > 0, 1.0, -1.0)
    return sgn * np.maximum(np.abs(w) - tau, 0.0)


# ---------------------------------------------------------------- DCT
def dct_matrix(n: int) -> np.ndarray:
    """Orthonormal DCT-II matrix C[k, m] = a_k cos(pi (2m + 1) k / (2n)),
    a_0 = sqrt(1/n), a_k = sqrt(2/n) otherwise (rows are the basis vectors)."""
    k = np.arange(n)[:, None].astype(np.float64)
    m = np.arange(n)[None, :].astype(np.float64)
    c = np.cos(math.pi * (2.0 * m + 1.0) * k / (2.0 * n))
    a = np.full((n, 1), math.sqrt(2.0 / n))
    a[0, 0] = math.sqrt(1.0 / n)
    return a * c


class DCT2D:
    """T x = C_{N1} x_s C_{N2}^T for every slice (2D transform per slice)."""

    name = "dct2d"

    def __init__(self, S: int, N1: int, N2: int):
        self.S, self.N1, self.N2 = S, N1, N2
        self.C1 = dct_matrix(N1)
        self.C2 = dct_matrix(N2)
        self.shape = (1, S, N1, N2)

    def T(self, x):
        return (self.C1 @ x @ self.C2.T)[None]

    def Tt(self, w):
        return self.C1.T @ w[0] @ self.C2

    def gram_symbol(self, N1, N2):
        """T^H T = I: the per-frequency symbol is 1."""
        return np.ones((N1, N2))


class DCT3D(DCT2D):
    """A single 3D transform over the cube (Section III-A: a 3D transform when
    the data are correlated along all three dimensions): the orthonormal
    DCT-II along the band axis applied to the 2D DCT of every slice,
    T x = C_S (C_{N1} x_s C_{N2}^T) with C_S acting on the slice index."""

    name = "dct3d"

    def __init__(self, S: int, N1: int, N2: int):
        super().__init__(S, N1, N2)
        self.CS = dct_matrix(S)

    def T(self, x):
        w2 = self.C1 @ x @ self.C2.T                        # (S, N1, N2)
        return np.tensordot(self.CS, w2, axes=(1, 0))[None]

    def Tt(self, w):
        w2 = np.tensordot(self.CS.T, w[0], axes=(1, 0))
        return self.C1.T @ w2 @ self.C2


# ---------------------------------------------------------------- wavelet (x) DCT
# Symmlet-8 scaling filter (Daubechies' least-asymmetric orthonormal wavelet
# with 8 vanishing moments; 16 taps, sum sqrt(2), unit energy).
SYM8 = np.array([
    -0.0033824159510061256, -0.0005421323317911481, 0.03169508781149298,
    0.007607487324917605, -0.1432942383508097, -0.061273359067658524,
    0.4813596512583722, 0.7771857517005235, 0.3644418948353314,
    -0.05194583810770904, -0.027219029917056003, 0.049137179673607506,
    0.003808752013890615, -0.01495225833704823, -0.0003029205147213668,
    0.0018899503327594609])


def qmf_highpass(h: np.ndarray) -> np.ndarray:
    """Wavelet filter of an orthonormal scaling filter: g[t] = (-1)^t h[L-1-t]."""
    L = len(h)
    return np.array([(-1.0) ** t * h[L - 1 - t] for t in range(L)])


def dwt1(x: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """One level of the periodized orthonormal DWT along `axis`:
    a[k] = sum_t h[t] x[(2k + t) mod N], d[k] = sum_t g[t] x[(2k + t) mod N];
    the output holds [a | d] along the axis."""
    g = qmf_highpass(h)
    xa = np.moveaxis(x, axis, -1)
    a = sum(h[t] * np.roll(xa, -t, axis=-1)[..., ::2] for t in range(len(h)))
    d = sum(g[t] * np.roll(xa, -t, axis=-1)[..., ::2] for t in range(len(h)))
    return np.moveaxis(np.concatenate([a, d], axis=-1), -1, axis)


def idwt1(c: np.ndarray, h: np.ndarray, axis: int) -> np.ndarray:
    """Adjoint (= inverse) of dwt1: x[n] = sum_k a[k] h[n - 2k] + d[k] g[n - 2k]
    (indices mod N)."""
    g = qmf_highpass(h)
    ca = np.moveaxis(c, axis, -1)
    n = ca.shape[-1]
    ua = np.zeros_like(ca)
    ud = np.zeros_like(ca)
    ua[..., ::2] = ca[..., : n // 2]
    ud[..., ::2] = ca[..., n // 2:]
    x = sum(h[t] * np.roll(ua, t, axis=-1) + g[t] * np.roll(ud, t, axis=-1)
            for t in range(len(h)))
    return np.moveaxis(x, -1, axis)


class WaveletDCT:
    """The Kronecker transform of Section V-A for the analysis prior: the 2D
    Symmlet-8 wavelet transform of every slice (periodized, `levels` levels,
    Mallat layout: each level transforms the low-pass corner of the previous
    one along both image axes) followed by the orthonormal DCT-II along the
    band axis. Orthonormal, so T^H T = I."""

    name = "wdct3d"

    def __init__(self, S: int, N1: int, N2: int, levels: int = 3):
        assert N1 % (1 << levels) == 0 and N2 % (1 << levels) == 0
        self.S, self.N1, self.N2, self.levels = S, N1, N2, levels
        self.h = SYM8
        self.CS = dct_matrix(S)
        self.shape = (1, S, N1, N2)

    def wavelet2(self, x):
        """2D DWT of every slice of x (S, N1, N2)."""
        c = np.array(x, dtype=np.float64, copy=True)
        r, q = self.N1, self.N2
        for _ in range(self.levels):
            blk = dwt1(dwt1(c[:, :r, :q], self.h, axis=2), self.h, axis=1)
            c[:, :r, :q] = blk
            r, q = r // 2, q // 2
        return c

    def iwavelet2(self, c):
        x = np.array(c, dtype=np.float64, copy=True)
        sizes = [(self.N1 >> l, self.N2 >> l) for l in range(self.levels)]
        for r, q in reversed(sizes):
            x[:, :r, :q] = idwt1(idwt1(x[:, :r, :q], self.h, axis=1), self.h, axis=2)
        return x

    def T(self, x):
        return np.tensordot(self.CS, self.wavelet2(x), axes=(1, 0))[None]

    def Tt(self, w):
        return self.iwavelet2(np.tensordot(self.CS.T, w[0], axes=(1, 0)))

    def gram_symbol(self, N1, N2):
        """T^H T = I: the per-frequency symbol is 1."""
        return np.ones((N1, N2))


class TV2D:
    """Anisotropic gradient per slice, circular forward differences:
    w[0] = x[n1 + 1, n2] - x[n1, n2],  w[1] = x[n1, n2 + 1] - x[n1, n2]."""

    name = "tv2d"

    def __init__(self, S: int, N1: int, N2: int):
        self.S, self.N1, self.N2 = S, N1, N2
        self.shape = (2, S, N1, N2)

    def T(self, x):
        w = np.empty((2,) + x.shape)
        w[0] = np.roll(x, -1, axis=1) - x
        w[1] = np.roll(x, -1, axis=2) - x
        return w

    def Tt(self, w):
        return (np.roll(w[0], 1, axis=1) - w[0]) + (np.roll(w[1], 1, axis=2) - w[1])

    def gram_symbol(self, N1, N2):
        """T^T T is the circular Laplacian; its DFT symbol is
        (2 - 2 cos w1) + (2 - 2 cos w2)."""
        w1 = 2.0 * math.pi * np.arange(N1)[:, None] / N1
        w2 = 2.0 * math.pi * np.arange(N2)[None, :] / N2
        return (2.0 - 2.0 * np.cos(w1)) + (2.0 - 2.0 * np.cos(w2))


class TV3D(TV2D):
    """TV2D plus a band-axis forward difference w[2][s] = x[s + 1] - x[s] for
    s < S - 1 and w[2][S - 1] = 0 (no wrap along the bands)."""

    name = "tv3d"

    def __init__(self, S: int, N1: int, N2: int):
        super().__init__(S, N1, N2)
        self.shape = (3, S, N1, N2)

    def T(self, x):
        w = np.zeros((3,) + x.shape)
        w[:2] = super().T(x)
        w[2, :-1] = x[1:] - x[:-1]
        return w

    def Tt(self, w):
        g = super().Tt(w[:2])
        q = w[2].copy()
        q[-1] = 0.0
        g[1:] += q[:-1]
        g -= q
        return g

    def band_laplacian(self):
        """D_s^T D_s for the band difference: the S x S path-graph Laplacian."""
        S = self.S
        L = np.zeros((S, S))
        for s in range(S - 1):
            L[s, s] += 1.0
            L[s + 1, s + 1] += 1.0
            L[s, s + 1] -= 1.0
            L[s + 1, s] -= 1.0
        return L


class Identity:
    """T = I: the analysis split used with isotropic TV (Phi(Tx) = TV(x) with
    T = I, Section III-A; per slice, or coupled along the slices); the
    t-update is then the TV proximal map."""

    name = "itv2d"

    def __init__(self, S: int, N1: int, N2: int):
        self.S, self.N1, self.N2 = S, N1, N2
        self.shape = (1, S, N1, N2)

    def T(self, x):
        return x[None].copy()

    def Tt(self, w):
        return w[0].copy()

    def gram_symbol(self, N1, N2):
        return np.ones((N1, N2))


def make_transform(kind: str, S: int, N1: int, N2: int, levels: int = 3):
    if kind == "wdct3d":
        return WaveletDCT(S, N1, N2, levels)
    return {"dct2d": DCT2D, "dct3d": DCT3D, "tv2d": TV2D, "tv3d": TV3D,
            "itv2d": Identity, "itv3d": Identity}[kind](S, N1, N2)


# ---------------------------------------------------------------- isotropic TV
def grad2(x: np.ndarray) -> np.ndarray:
    """Circular forward differences of every slice, shape (2,) + x.shape."""
    return np.stack([np.roll(x, -1, axis=-2) - x, np.roll(x, -1, axis=-1) - x])


def div2(p: np.ndarray) -> np.ndarray:
    """Discrete divergence, the negative adjoint of grad2:
    div p = (p0[n1] - p0[n1 - 1]) + (p1[n2] - p1[n2 - 1])."""
    return (p[0] - np.roll(p[0], 1, axis=-2)) + (p[1] - np.roll(p[1], 1, axis=-1))


def tv_iso(x: np.ndarray) -> float:
    """Isotropic TV, sum over pixels and slices of |grad x| (Euclidean)."""
    g = grad2(x)
    return float(np.sum(np.sqrt(g[0] ** 2 + g[1] ** 2)))


def chambolle(f: np.ndarray, mu: float, p: np.ndarray, iters: int, tau: float = 0.125):
    """Chambolle's projection algorithm for the isotropic-TV proximal map
    argmin_t 1/2 ||t - f||^2 + mu TV(t), every slice separately:
        p <- (p + tau grad(div p - f / mu)) / (1 + tau |grad(div p - f / mu)|),
    t = f - mu div p; tau <= 1/8 guarantees convergence. Starts from the dual
    p given (shape (2,) + f.shape) and returns (t, p)."""
    p = p.copy()
    for _ in range(iters):
        g = grad2(div2(p) - f / mu)
        nrm = np.sqrt(g[0] ** 2 + g[1] ** 2)
        p = (p + tau * g) / (1.0 + tau * nrm)
    return f - mu * div2(p), p


# ------------------------------------------------- isotropic TV coupled along the slices
def grad3(x: np.ndarray) -> np.ndarray:
    """Circular forward differences along both image axes and the forward
    difference along the slices (none after the last slice: that component
    is 0 there), shape (3,) + x.shape."""
    gb = np.zeros_like(x)
    gb[:-1] = x[1:] - x[:-1]
    return np.stack([np.roll(x, -1, axis=-2) - x, np.roll(x, -1, axis=-1) - x, gb])


def div3(p: np.ndarray) -> np.ndarray:
    """Discrete divergence, the negative adjoint of grad3: div2 of the image
    components plus p2[s] - p2[s - 1] along the slices (p2[-1] = 0; the last
    slice's p2, which grad3 never fills, is read as 0)."""
    b = p[2].copy()
    b[-1] = 0.0
    db = b.copy()
    db[1:] -= b[:-1]
    return div2(p[:2]) + db


def tv_iso3(x: np.ndarray) -> float:
    """Isotropic TV of the whole cube, sum over voxels of |grad3 x|."""
    g = grad3(x)
    return float(np.sum(np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)))


def chambolle3(f: np.ndarray, mu: float, p: np.ndarray, iters: int, tau: float = 1.0 / 12.0):
    """Chambolle's projection algorithm for the proximal map of the isotropic
    TV coupled along the slices, argmin_t 1/2 ||t - f||^2 + mu TV3(t):
        p <- (p + tau grad3(div3 p - f / mu)) / (1 + tau |grad3(div3 p - f / mu)|),
    t = f - mu div3 p. ||div3||^2 <= 12 (two circular axes and a path along
    the slices, each <= 4), so tau <= 1/12 keeps Chambolle's convergence
    argument. Starts from the dual p given (shape (3,) + f.shape) and
    returns (t, p)."""
    p = p.copy()
    for _ in range(iters):
        g = grad3(div3(p) - f / mu)
        nrm = np.sqrt(g[0] ** 2 + g[1] ** 2 + g[2] ** 2)
        p = (p + tau * g) / (1.0 + tau * nrm)
    return f - mu * div3(p), p


# ---------------------------------------------------------------- patches
class Patches:
    """Q x Q x S patches spanning all bands (Eq. patch_based with T = S),
    taken circularly at positions (i*st, j*st), i < N1/st, j < N2/st.

    Patch vector layout: element s*Q*Q + a*Q + b is
    x[s, (i*st + a) mod N1, (j*st + b) mod N2]; patch index j = i*(N2/st) + j.
    With st dividing Q, every pixel lies in (Q/st)^2 patches, so
    P^T P = (Q/st)^2 I (the constant t of Eq. solx_synt)."""

    def __init__(self, S: int, N1: int, N2: int, Q: int, st: int):
        assert N1 % st == 0 and N2 % st == 0
        self.S, self.N1, self.N2, self.Q, self.st = S, N1, N2, Q, st
        self.J1, self.J2 = N1 // st, N2 // st
        self.J = self.J1 * self.J2
        self.n = Q * Q * S
        s, a, b = np.meshgrid(np.arange(S), np.arange(Q), np.arange(Q), indexing="ij")
        self._s, self._a, self._b = s.ravel(), a.ravel(), b.ravel()

    def _index(self):
        """Row / column index of every patch element, shape (n, J)."""
        if not hasattr(self, "_rows"):
            i = np.repeat(np.arange(self.J1), self.J2)          # patch row of j
            j = np.tile(np.arange(self.J2), self.J1)            # patch column of j
            self._rows = (i[None, :] * self.st + self._a[:, None]) % self.N1
            self._cols = (j[None, :] * self.st + self._b[:, None]) % self.N2
        return self._rows, self._cols

    def extract(self, x: np.ndarray) -> np.ndarray:
        """X = [P_1 x | ... | P_J x], shape (n, J)."""
        rows, cols = self._index()
        return x[self._s[:, None], rows, cols]

    def adjoint(self, X: np.ndarray) -> np.ndarray:
        """sum_j P_j^T X[:, j] (overlap-add of patches back onto the grid)."""
        rows, cols = self._index()
        x = np.zeros((self.S, self.N1, self.N2))
        np.add.at(x, (np.broadcast_to(self._s[:, None], rows.shape), rows, cols), X)
        return x

    @property
    def c_P(self) -> float:
        return float((self.Q // self.st) ** 2)


# ---------------------------------------------------------------- conv dictionary
def filter_on_grid(d: np.ndarray, N1: int, N2: int) -> np.ndarray:
    """Place an L x L filter on the N1 x N2 torus, centred at [0, 0]: tap
    (a, b) sits at offset (a - L//2, b - L//2)."""
    L = d.shape[0]
    h = np.zeros((N1, N2))
    for a in range(L):
        for b in range(L):
            h[(a - L // 2) % N1, (b - L // 2) % N2] += d[a, b]
    return h


class ConvDict2D:
    """Common convolutional dictionary for every band (2D-correlation variant of
    Eq. conv_dic): band s is approximated by sum_m d_m * z_{m,s}; P = I."""

    def __init__(self, filters: np.ndarray, S: int, N1: int, N2: int):
        self.M = filters.shape[0]
        self.S, self.N1, self.N2 = S, N1, N2
        self.h = np.stack([filter_on_grid(f, N1, N2) for f in filters])

    def synth(self, z: np.ndarray) -> np.ndarray:
        """D~ z, z of shape (M, S, N1, N2) -> (S, N1, N2), spatial convolutions."""
        out = np.zeros((self.S, self.N1, self.N2))
        for m in range(self.M):
            for s in range(self.S):
                out[s] += conv_circ(z[m, s], self.h[m])
        return out

    def analysis(self, x: np.ndarray) -> np.ndarray:
        """D~^T x -> (M, S, N1, N2), spatial correlations."""
        z = np.empty((self.M, self.S, self.N1, self.N2))
        for m in range(self.M):
            for s in range(self.S):
                z[m, s] = corr_circ(x[s], self.h[m])
        return z

    def spectra(self) -> np.ndarray:
        """theta_m = 2D DFT of the grid-placed filters, shape (M, N1, N2)."""
        return np.fft.fft2(self.h)


class ConvDict3D:
    """Convolutional dictionary with 3D filters for data correlated along the
    bands too (Eq. conv_dic with 3D signals; Section IV-B writes each filter's
    convolution matrix as diagonal in the 3D DFT): x = sum_m d_m (*) z_m, a
    circular 3D convolution over (band, n1, n2) of the S x N1 x N2 code z_m
    with the S x L x L filter d_m. Band tap s' sits at band offset s' and
    spatial tap (a, b) at offset (a - L//2, b - L//2); P = I."""

    def __init__(self, filters: np.ndarray, S: int, N1: int, N2: int):
        M, Sf = filters.shape[:2]
        assert Sf == S, "3D filters span the S bands"
        self.M = M
        self.S, self.N1, self.N2 = S, N1, N2
        self.h = np.stack([np.stack([filter_on_grid(filters[m, sp], N1, N2) for sp in range(S)])
                           for m in range(M)])                   # (M, S, N1, N2)

    def synth(self, z: np.ndarray) -> np.ndarray:
        """D~ z, z of shape (M, S, N1, N2) -> (S, N1, N2), spatial convolutions:
        x[s] = sum_m sum_s' h_m[s'] * z_m[(s - s') mod S]."""
        out = np.zeros((self.S, self.N1, self.N2))
        for m in range(self.M):
            for s in range(self.S):
                for sp in range(self.S):
                    out[s] += conv_circ(z[m, (s - sp) % self.S], self.h[m, sp])
        return out

    def analysis(self, x: np.ndarray) -> np.ndarray:
        """D~^T x -> (M, S, N1, N2): z_m[s] = sum_s' corr(x[(s + s') mod S], h_m[s'])."""
        z = np.zeros((self.M, self.S, self.N1, self.N2))
        for m in range(self.M):
            for s in range(self.S):
                for sp in range(self.S):
                    z[m, s] += corr_circ(x[(s + sp) % self.S], self.h[m, sp])
        return z

    def spectra(self) -> np.ndarray:
        """theta_m = 3D DFT of the grid-placed filters, shape (M, S, N1, N2)
        (band frequency first)."""
        return np.fft.fftn(self.h, axes=(1, 2, 3))


def gradient_filters_2d(N1: int, N2: int):
    """r_1, r_2 of Eq. DL_PriorHP_conv for 2D correlations, as kernels on the
    N1 x N2 torus: circular forward differences, (r_i * z)[n] = z[n + e_i] - z[n]
    (tap -1 at offset 0, +1 at offset -e_i)."""
    r1 = np.zeros((N1, N2))
    r2 = np.zeros((N1, N2))
    r1[0, 0] = r2[0, 0] = -1.0
    r1[-1 % N1, 0] = 1.0
    r2[0, -1 % N2] = 1.0
    return r1, r2


def tikhonov_symbol(N1: int, N2: int) -> np.ndarray:
    """Per-frequency symbol of sum_i R_i^H R_i: sum_i |DFT(r_i)|^2."""
    r1, r2 = gradient_filters_2d(N1, N2)
    return np.abs(np.fft.fft2(r1)) ** 2 + np.abs(np.fft.fft2(r2)) ** 2
