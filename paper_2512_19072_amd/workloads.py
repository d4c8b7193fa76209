"""Seeded synthetic beam images for the FOT hot path.

Section 4 of the paper measures FOT on a two-Gaussian input beam and target images
that are printed only as figures (Fig. 1, Fig. 3, Fig. 4), so every workload here is
synthetic: amplitudes ``g`` (input plane) and ``G`` (Fourier plane) on n x n grids,
generated in float64 on the host from ``numpy.random.default_rng(seed)``.

This module holds no arithmetic of the method: it draws pictures and returns
amplitudes.  Normalisation, logarithms, kernels and potentials are computed by the
solver under test and, independently, by the oracle.  Pixel lengths are given for a
1024-pixel grid and scaled by ``n / 1024`` so that smaller grids keep the same shapes
(``n=1024`` reproduces the stated sizes exactly).

Workloads (index = position in :data:`WORKLOADS`):

0. ``gauss_to_disk``     64 x 64, Gaussian input (sigma 10 px) -> flat-top disk of
                          radius 20 px with exact zeros outside; eps 1e-2, 200 iters.
1. ``twogauss_to_shapes`` 1024 x 1024, 0.6/0.4 sum of Gaussians (sigma 150, 90 px,
                          second centre offset by (+60, -40) px) -> union of 8 random
                          ellipses and 2 random rings, intensity 1 inside, 1e-6 outside;
                          eps 5e-3, 200 iters (FP32).
2. same images as 1, low-precision operand forms (BF16 / FP16).
3. ``speckle_to_lattice`` 2048 x 2048, elliptical Gaussian (sigma 500 x 350 px) with 5 %
                          log-normal speckle -> 16 x 16 lattice of Gaussian spots
                          (sigma 4 px, pitch 64 px) with U[0.8, 1.2] amplitudes; eps
                          annealed geometrically 5e-2 -> 2e-3 over 400 iters.
4. ``gauss_to_ellipses`` 512 x 512, Gaussian input (sigma 80 px) -> 8 targets (seeds
                          0..7), each the union of 4 random ellipses with a 1e-6 floor;
                          eps 5e-3, 100 iters, adjoint with checkpoints every 10.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from typing import Optional

import numpy as np

__all__ = [
    "grid", "gaussian", "ellipse_mask", "ring_mask",
    "gauss_to_disk", "twogauss_to_shapes", "speckle_to_lattice", "gauss_to_ellipses",
    "anneal_schedule", "Workload", "WORKLOADS", "workload",
]


def grid(n: int):
    """Integer pixel index arrays (j, k) of shape (n, n); j is the row (x axis)."""
    j = np.arange(n, dtype=np.float64)[:, None]
    k = np.arange(n, dtype=np.float64)[None, :]
    return np.broadcast_to(j, (n, n)), np.broadcast_to(k, (n, n))


def gaussian(n, cj, ck, sj, sk=None):
    """Amplitude exp(-(j-cj)^2/(2 sj^2) - (k-ck)^2/(2 sk^2)) on the n x n grid."""
    sk = sj if sk is None else sk
    j, k = grid(n)
    return np.exp(-((j - cj) ** 2) / (2.0 * sj * sj) - ((k - ck) ** 2) / (2.0 * sk * sk))


def ellipse_mask(n, cj, ck, aj, ak, theta):
    """Boolean mask of a filled ellipse with semi-axes (aj, ak) rotated by theta."""
    j, k = grid(n)
    dj, dk = j - cj, k - ck
    c, s = math.cos(theta), math.sin(theta)
    u = dj * c + dk * s
    v = -dj * s + dk * c
    return (u / aj) ** 2 + (v / ak) ** 2 <= 1.0


def ring_mask(n, cj, ck, radius, width):
    """Boolean mask of an annulus of the given centre radius and full width."""
    j, k = grid(n)
    r = np.sqrt((j - cj) ** 2 + (k - ck) ** 2)
    return np.abs(r - radius) <= 0.5 * width


def gauss_to_disk(n: int = 64):
    """Workload 0: centred Gaussian (sigma 10 px at n=64) -> disk (radius 20 px at n=64).

    The target intensity is exactly zero outside the disk, which exercises zero-mass
    pixels (infinite potentials).  Lengths scale with n / 64 here because the
    workload is defined on a 64-pixel grid.
    """
    s = n / 64.0
    c = n // 2
    g = gaussian(n, c, c, 10.0 * s)
    j, k = grid(n)
    G = (((j - c) ** 2 + (k - c) ** 2) <= (20.0 * s) ** 2).astype(np.float64)
    return g, G


def twogauss_to_shapes(n: int = 1024, seed: int = 0):
    """Workload 1/2: asymmetric two-Gaussian input -> 8 ellipses + 2 rings.

    Random draws, in order: 8 x (cj, ck, aj, ak, theta) then 2 x (R, w, cj, ck).
    """
    s = n / 1024.0
    c = n // 2
    g = 0.6 * gaussian(n, c, c, 150.0 * s) + 0.4 * gaussian(n, c + 60.0 * s, c - 40.0 * s, 90.0 * s)
    rng = np.random.default_rng(seed)
    inside = np.zeros((n, n), dtype=bool)
    for _ in range(8):
        cj, ck = rng.uniform(0.25 * n, 0.75 * n, size=2)
        aj, ak = rng.uniform(50.0 * s, 300.0 * s, size=2)
        th = rng.uniform(0.0, math.pi)
        inside |= ellipse_mask(n, cj, ck, aj, ak, th)
    for _ in range(2):
        R = rng.uniform(50.0 * s, 300.0 * s)
        w = rng.uniform(10.0 * s, 30.0 * s)
        cj, ck = rng.uniform(0.35 * n, 0.65 * n, size=2)
        inside |= ring_mask(n, cj, ck, R, w)
    intensity = np.where(inside, 1.0, 1e-6)
    return g, np.sqrt(intensity)


def speckle_to_lattice(n: int = 2048, seed: int = 0):
    """Workload 3: speckled elliptical Gaussian -> 16 x 16 lattice of Gaussian spots.

    Random draws, in order: n*n standard normals for the speckle, then 256 spot
    amplitudes U[0.8, 1.2] (row-major over the lattice).
    """
    s = n / 2048.0
    c = n // 2
    rng = np.random.default_rng(seed)
    z = rng.standard_normal((n, n))
    g = gaussian(n, c, c, 500.0 * s, 350.0 * s) * np.exp(0.05 * z)
    amp = rng.uniform(0.8, 1.2, size=(16, 16))
    pitch = 64.0 * s
    centres = c + (np.arange(16) - 7.5) * pitch
    sig = 4.0 * s
    jj = np.arange(n, dtype=np.float64)
    # each spot is separable, so the lattice is a sum of outer products
    ej = np.exp(-((jj[None, :] - centres[:, None]) ** 2) / (2.0 * sig * sig))   # [16][n]
    G = ej.T @ amp @ ej                                                          # [n][n]
    return g, G


def gauss_to_ellipses(n: int = 512, n_targets: int = 8):
    """Workload 4: Gaussian input (sigma 80 px at n=512) -> n_targets ellipse unions.

    Target b uses ``default_rng(b)`` and draws 4 x (cj, ck, aj, ak, theta); lengths
    scale with n / 512.
    """
    s = n / 512.0
    c = n // 2
    g = gaussian(n, c, c, 80.0 * s)
    Gs = np.empty((n_targets, n, n))
    for b in range(n_targets):
        rng = np.random.default_rng(b)
        inside = np.zeros((n, n), dtype=bool)
        for _ in range(4):
            cj, ck = rng.uniform(0.25 * n, 0.75 * n, size=2)
            aj, ak = rng.uniform(20.0 * s, 120.0 * s, size=2)
            th = rng.uniform(0.0, math.pi)
            inside |= ellipse_mask(n, cj, ck, aj, ak, th)
        Gs[b] = np.sqrt(np.where(inside, 1.0, 1e-6))
    return g, Gs


def fd_pixels(n: int, target: int, count: int = 64):
    """Pixel indices (flat, row-major) at which target ``target`` is finite-differenced."""
    rng = np.random.default_rng(1000 + target)
    return rng.choice(n * n, size=count, replace=False)


def anneal_schedule(eps0: float, eps1: float, iters: int):
    """Geometric schedule eps_t = eps0 (eps1/eps0)^(t/(iters-1)), t = 0..iters-1."""
    if iters == 1:
        return np.array([eps0], dtype=np.float64)
    t = np.arange(iters, dtype=np.float64)
    return eps0 * (eps1 / eps0) ** (t / (iters - 1))


@dataclass
class Workload:
    name: str
    n: int
    iters: int
    eps: np.ndarray
    precisions: tuple
    batch: int = 1
    checkpoint_every: int = 0
    make: Optional[object] = field(default=None, repr=False)

    def images(self, n: Optional[int] = None):
        """(g [n][n], G [batch][n][n]) amplitudes, at the workload's own n by default."""
        g, G = self.make(self.n if n is None else n)
        if G.ndim == 2:
            G = G[None]
        return g, G


WORKLOADS = [
    Workload("gauss_to_disk", 64, 200, np.array([1e-2]), ("f64",), make=gauss_to_disk),
    Workload("twogauss_to_shapes", 1024, 200, np.array([5e-3]), ("f32",), make=twogauss_to_shapes),
    Workload("twogauss_to_shapes_lowp", 1024, 200, np.array([5e-3]), ("bf16", "f16"),
             make=twogauss_to_shapes),
    Workload("speckle_to_lattice", 2048, 400, anneal_schedule(5e-2, 2e-3, 400), ("f32", "bf16"),
             make=speckle_to_lattice),
    Workload("gauss_to_ellipses", 512, 100, np.array([5e-3]), ("f32",), batch=8,
             checkpoint_every=10, make=gauss_to_ellipses),
]


def workload(i: int) -> Workload:
    return WORKLOADS[i]
