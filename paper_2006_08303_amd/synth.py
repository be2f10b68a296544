"""Seeded synthetic inputs shaped like the paper's spectral-imaging workloads.

This module only draws random numbers and paints test images and blur kernels.
It holds none of the reconstruction method's arithmetic (no forward model, no
transform, no solve): both the CPU oracle and the GPU library consume what it
produces, so it must stay free of either side's code.

Workloads (the paper's datasets are not available, so these stand in for them):

* ``rects``   -- piecewise-constant images: random axis-aligned rectangles per
                 band, values in [0, 1] (small-problem case, K = S = 2, 64x64).
* ``smooth``  -- band-correlated smooth fields plus random straight edges,
                 mixed across bands by a random row-stochastic matrix and
                 min-max scaled to [0, 1] (spectral-imaging case, K = S = 3).

Blur kernels follow the paper's spectral-imaging setup (Section V: each
measurement focuses one band and defocuses the others): Gaussian kernels with
random widths, or defocus disks whose radius grows with the distance between
the measurement index and the band index. Kernels are unit-sum, stored
unshifted (origin at [0, 0]) and wrapped circularly on the N1 x N2 grid.

All generators use NumPy's PCG64 with ``seed = 1000 * config + index``.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = [
    "rng_for",
    "rect_images",
    "smooth_images",
    "gaussian_psfs",
    "disk_psfs",
    "unit_noise",
    "random_unit_atoms",
    "random_unit_filters",
    "random_unit_filters_3d",
    "problem",
]


def rng_for(config: int, index: int = 0) -> np.random.Generator:
    """PCG64 generator with the seed rule ``1000 * config + index``."""
    return np.random.Generator(np.random.PCG64(1000 * int(config) + int(index)))


def rect_images(rng: np.random.Generator, S: int, N1: int, N2: int,
                n_rect: int = 10, side=(4, 32)) -> np.ndarray:
    """S bands, each with ``n_rect`` axis-aligned rectangles painted over 0.

    Sides are uniform integers in [side[0], side[1]], values uniform in [0, 1],
    positions uniform (rectangles wrap around the torus)."""
    x = np.zeros((S, N1, N2), dtype=np.float64)
    for s in range(S):
        for _ in range(n_rect):
            h = int(rng.integers(side[0], side[1] + 1))
            w = int(rng.integers(side[0], side[1] + 1))
            r0 = int(rng.integers(0, N1))
            c0 = int(rng.integers(0, N2))
            val = float(rng.uniform(0.0, 1.0))
            rows = (r0 + np.arange(h)) % N1
            cols = (c0 + np.arange(w)) % N2
            x[s][np.ix_(rows, cols)] = val
    return x


def _gauss_smooth_periodic(field: np.ndarray, sigma: float) -> np.ndarray:
    """Circular Gaussian smoothing of a 2D field (generator-side helper)."""
    n1, n2 = field.shape
    f1 = np.fft.fftfreq(n1)[:, None]
    f2 = np.fft.fftfreq(n2)[None, :]
    g = np.exp(-2.0 * (math.pi * sigma) ** 2 * (f1 ** 2 + f2 ** 2))
    return np.real(np.fft.ifft2(np.fft.fft2(field) * g))


def smooth_images(rng: np.random.Generator, S: int, N1: int, N2: int,
                  n_edges: int = 12) -> np.ndarray:
    """Band-correlated smooth random fields with straight edges, in [0, 1].

    Per latent band: white noise smoothed with a circular Gaussian of width
    N/32, rescaled to unit variance, plus ``n_edges`` random half-plane steps
    with amplitudes uniform in [-0.5, 0.5]. Bands are then mixed by a random
    row-stochastic matrix (0.6 I + 0.4 U[0,1], rows normalised) and the whole
    cube is min-max scaled to [0, 1]."""
    lat = np.empty((S, N1, N2), dtype=np.float64)
    ii = np.arange(N1, dtype=np.float64)[:, None]
    jj = np.arange(N2, dtype=np.float64)[None, :]
    sig = max(N1, N2) / 32.0
    for s in range(S):
        f = _gauss_smooth_periodic(rng.standard_normal((N1, N2)), sig)
        f = (f - f.mean()) / (f.std() + 1e-30)
        for _ in range(n_edges):
            ang = rng.uniform(0.0, 2.0 * math.pi)
            off = rng.uniform(-0.5, 0.5) * min(N1, N2)
            amp = rng.uniform(-0.5, 0.5)
            d = (ii - N1 / 2.0) * math.cos(ang) + (jj - N2 / 2.0) * math.sin(ang)
            f = f + amp * (d > off)
        lat[s] = f
    mix = 0.6 * np.eye(S) + 0.4 * rng.uniform(0.0, 1.0, size=(S, S))
    mix /= mix.sum(axis=1, keepdims=True)
    x = np.einsum("ab,bij->aij", mix, lat)
    lo, hi = x.min(), x.max()
    return (x - lo) / (hi - lo)


def _wrap_kernel(N1: int, N2: int, taps: dict) -> np.ndarray:
    h = np.zeros((N1, N2), dtype=np.float64)
    for (a, b), v in taps.items():
        h[a % N1, b % N2] += v
    return h


def gaussian_psfs(rng: np.random.Generator, K: int, S: int, N1: int, N2: int,
                  sigma_range=(1.0, 4.0)) -> np.ndarray:
    """K x S Gaussian blur kernels, widths uniform in ``sigma_range``.

    Each kernel is sampled on the integer offsets within radius ceil(4 sigma),
    normalised to unit sum and wrapped onto the grid with its centre at [0, 0]."""
    psf = np.zeros((K, S, N1, N2), dtype=np.float64)
    for k in range(K):
        for s in range(S):
            sg = float(rng.uniform(*sigma_range))
            r = int(math.ceil(4.0 * sg))
            a = np.arange(-r, r + 1)
            g = np.exp(-(a[:, None] ** 2 + a[None, :] ** 2) / (2.0 * sg * sg))
            g /= g.sum()
            taps = {(int(a[i]), int(a[j])): g[i, j]
                    for i in range(len(a)) for j in range(len(a))}
            psf[k, s] = _wrap_kernel(N1, N2, taps)
    return psf


def disk_radius(k: int, s: int, K: int, S: int, r_max: float = 8.0) -> float:
    """Defocus radius growing with |k/(K-1) - s/(S-1)| (0 on the focused band)."""
    a = k / (K - 1) if K > 1 else 0.0
    b = s / (S - 1) if S > 1 else 0.0
    return r_max * abs(a - b)


def disk_psfs(K: int, S: int, N1: int, N2: int, r_max: float = 8.0) -> np.ndarray:
    """K x S uniform defocus disks (radius 0 is a delta), unit sum, origin [0,0]."""
    psf = np.zeros((K, S, N1, N2), dtype=np.float64)
    for k in range(K):
        for s in range(S):
            r = disk_radius(k, s, K, S, r_max)
            R = int(math.floor(r))
            taps = {}
            for a in range(-R, R + 1):
                for b in range(-R, R + 1):
                    if a * a + b * b <= r * r + 1e-9:
                        taps[(a, b)] = 1.0
            tot = float(len(taps))
            psf[k, s] = _wrap_kernel(N1, N2, {kk: v / tot for kk, v in taps.items()})
    return psf


def unit_noise(rng: np.random.Generator, K: int, N1: int, N2: int) -> np.ndarray:
    """Standard normal noise, one plane per measurement (scaled by the caller)."""
    return rng.standard_normal((K, N1, N2))


def random_unit_atoms(rng: np.random.Generator, n: int, A: int) -> np.ndarray:
    """Dictionary with A Gaussian random atoms of length n, unit l2 norm.

    Returned as an (n, A) array: column a is atom a."""
    d = rng.standard_normal((n, A))
    d /= np.linalg.norm(d, axis=0, keepdims=True)
    return d


def random_unit_filters(rng: np.random.Generator, M: int, L: int) -> np.ndarray:
    """M random L x L filters with unit l2 norm, shape (M, L, L)."""
    f = rng.standard_normal((M, L, L))
    f /= np.linalg.norm(f.reshape(M, -1), axis=1)[:, None, None]
    return f

def random_unit_filters_3d(rng: np.random.Generator, M: int, S: int, L: int) -> np.ndarray:
    """M random S x L x L filters (standard normal taps), each scaled to unit
    l2 norm; float32-representable values as float64."""
    f = rng.standard_normal((M, S, L, L))
    f /= np.linalg.norm(f.reshape(M, -1), axis=1)[:, None, None, None]
    return f.astype(np.float32).astype(np.float64)


def problem(kind: str, N: int, K: int, S: int, seed_config: int,
            f32: bool = True):
    """Image cube, blur kernels and unit noise for one named workload.

    ``kind`` is ``"rects_gauss"`` (rectangles + Gaussian kernels) or
    ``"smooth_disk"`` (smooth fields + defocus disks). When ``f32`` is set the
    arrays are rounded to float32 and returned as float64 copies of those
    values, so that both sides of a comparison see identical inputs."""
    if kind == "rects_gauss":
        x = rect_images(rng_for(seed_config, 0), S, N, N)
        psf = gaussian_psfs(rng_for(seed_config, 1), K, S, N, N)
    elif kind == "smooth_disk":
        x = smooth_images(rng_for(seed_config, 0), S, N, N)
        psf = disk_psfs(K, S, N, N)
    else:
        raise ValueError(f"unknown workload kind {kind!r}")
    noise = unit_noise(rng_for(seed_config, 2), K, N, N)
    if f32:
        x = x.astype(np.float32).astype(np.float64)
        psf = psf.astype(np.float32).astype(np.float64)
        noise = noise.astype(np.float32).astype(np.float64)
    return x, psf, noise
