"""FP64 CPU reference of cFOT: the Sinkhorn iteration with Lambda . X . Lambda evaluated as 1-D
linear convolutions by FFT (Sec. 3, convolutional speedup, Eq. 11).

TEST INFRASTRUCTURE ONLY (like fot_oracle): imported by the tests, never by the library or its
binding, and importing nothing from them.

The iteration is the one of fot_oracle.solve_sep (Eq. 7-8 in log form, potentials carried across
an eps schedule); only the contraction differs: each row of exp(X - rowmax) is convolved with
lambda_j = exp(-j^2 / (2 n^2 eps)), j = -(n-1) .. n-1, through numpy's FFT of length
N = 2^ceil(log2(2n - 1)) (zero padding makes the circular convolution equal to the linear one on
the n outputs), and a result that rounding has made non-positive has logarithm -inf.  It exists to
show, independently of the GPU, what FFT convolution in FP64 does: it agrees with the exact
separable products while the convolution values stay well above 1e-16 of their row's largest, and
loses the small ones (non-finite potentials) once eps is small enough, the instability the paper
reports for cFOT (Sec. 4).
"""
from __future__ import annotations

import math

import numpy as np

from .fot_oracle import normalise

__all__ = ["fft_length", "lambda_transform", "conv_log_rows", "solve_conv"]


def fft_length(n: int) -> int:
    N = 1
    while N < 2 * n - 1:
        N *= 2
    return N


def lambda_transform(n: int, N: int, eps: float) -> np.ndarray:
    """DFT of lambda's circular extension (real: lambda is even)."""
    lc = np.zeros(N)
    for d in range(n):
        lc[d] = math.exp(-d * d / (2.0 * n * n * eps))
        if d:
            lc[N - d] = lc[d]
    return np.fft.fft(lc).real


def conv_log_rows(L: np.ndarray, lam_hat: np.ndarray) -> np.ndarray:
    """ln sum_M exp(L[r][M]) lambda(M - k) for every row r and k < n, by FFT, with the row maximum
    as shift (-inf rows stay -inf; non-positive results give -inf)."""
    rows, n = L.shape
    N = lam_hat.size
    m = np.max(L, axis=1, keepdims=True)
    empty = ~np.isfinite(m)
    s = np.where(empty, 0.0, m)
    x = np.zeros((rows, N))
    x[:, :n] = np.exp(L - s)
    y = np.fft.ifft(np.fft.fft(x, axis=1) * lam_hat[None, :], axis=1).real[:, :n]
    with np.errstate(divide="ignore", invalid="ignore"):
        out = np.where(y > 0, s + np.log(np.where(y > 0, y, 1.0)), -np.inf)
    return np.where(empty, -np.inf, out)


def solve_conv(g: np.ndarray, G: np.ndarray, eps, iters: int):
    """Potentials (f, psi) after `iters` iterations with FFT convolutions; eps a scalar or a
    per-iteration schedule."""
    a, b = normalise(g), normalise(G)
    with np.errstate(divide="ignore"):
        la, lb = np.log(a), np.log(b)
    n = a.shape[0]
    e = np.broadcast_to(np.asarray(eps, dtype=np.float64), (iters,))
    N = fft_length(n)
    f = np.full((n, n), e[0] * math.log(1.0 / (n * n)))   # u = V = 1/n^2, as in solve_sep
    psi = f.copy()
    lam_hat, lam_eps = None, None
    for t in range(iters):
        ep = float(e[t])
        if lam_eps != ep:
            lam_hat, lam_eps = lambda_transform(n, N, ep), ep
        # Eq. 7: ln S = ln(Lambda . V . Lambda), rows (axis 1) then columns (axis 0)
        lnS = conv_log_rows(conv_log_rows(psi / ep, lam_hat).T, lam_hat).T
        with np.errstate(invalid="ignore"):
            f = np.where(la > -np.inf, ep * (la - lnS), -np.inf)
        # Eq. 8
        lnSp = conv_log_rows(conv_log_rows(f / ep, lam_hat).T, lam_hat).T
        with np.errstate(invalid="ignore"):
            psi = np.where(lb > -np.inf, ep * (lb - lnSp), -np.inf)
    return f, psi
