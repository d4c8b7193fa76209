"""FP64 CPU oracle of the output-beam evaluation and of Gerchberg-Saxton polishing.

TEST INFRASTRUCTURE ONLY (like fot_oracle): imported by the tests and the benchmark's CPU
leg, never by the library or its binding, and importing nothing from them.

What is computed:

* the output beam of a phase: the Fraunhofer pattern |F[g e^{2 pi i phi}]|^2 of Eq. 1, with F
  the discrete Fourier transform between the two centred grids of Sec. 2,
      F[f]_LM = sum_jk f_jk exp(-2 pi i (x_j X_L + y_k Y_M)),  x_j X_L = (j - c)(L - c) / n,
  c = floor(n / 2), written out as the matrix product W f W^T with W_Lj = exp(-2 pi i
  (L - c)(j - c) / n);
* the L1 intensity loss of Sec. 4 (the Fig. 3 metric): the L1 norm of the difference between
  the output intensity and the target intensity G^2;
* Gerchberg-Saxton iterations (the textbook polishing step that Sec. 4 names), starting from a
  given phase.

Readings (the paper gives the metric by name, not its conventions):

B1  The transform's sign is exp(-2 pi i x X): a phase whose gradient is dphi/dx = X0 then
    sends light to X = X0, as the transport map of Eq. 4-5 does (with the opposite sign the
    beam would land at -X0).
B2  Both intensities are compared at unit total power: I = |F|^2 / sum |F|^2, which equals
    |F|^2 / (n^2 sum g^2) by Parseval, and b = G^2 / sum G^2.
B3  One Gerchberg-Saxton round: f = g e^{2 pi i phi}; F = W f W^T; F <- G F / |F| (phase 0
    where F = 0); f = conj(W) F conj(W)^T (the inverse up to the factor 1/n^2, which does not
    change a phase); phi = arg(f) / (2 pi) in (-1/2, 1/2].
"""
from __future__ import annotations

import numpy as np

__all__ = ["dft_matrix", "output_field", "output_beam", "l1_loss", "polish_gs"]


def dft_matrix(n: int) -> np.ndarray:
    """W[L, j] = exp(-2 pi i (L - c)(j - c) / n), c = floor(n/2) (B1).  The integer product is
    reduced mod n before the exponential, so every entry is a root of unity to FP64 rounding."""
    c = n // 2
    idx = np.arange(n) - c
    r = np.mod(np.outer(idx, idx), n)
    return np.exp(-2j * np.pi * r / n)


def output_field(g: np.ndarray, phase: np.ndarray) -> np.ndarray:
    """F[g e^{2 pi i phi}] on the target grid (Eq. 1)."""
    g = np.asarray(g, dtype=np.float64)
    W = dft_matrix(g.shape[0])
    f = g * np.exp(2j * np.pi * np.asarray(phase, dtype=np.float64))
    return W @ f @ W.T


def output_beam(g: np.ndarray, phase: np.ndarray) -> np.ndarray:
    """Unit-power output intensity |F|^2 / sum |F|^2 (B2)."""
    F = output_field(g, phase)
    I = np.abs(F) ** 2
    return I / np.sum(I)


def l1_loss(g: np.ndarray, phase: np.ndarray, G: np.ndarray) -> float:
    """sum_LM |I_LM - G^2_LM / sum G^2| (the L1 intensity loss of Sec. 4, read as B2)."""
    I = output_beam(g, phase)
    b = np.asarray(G, dtype=np.float64) ** 2
    return float(np.sum(np.abs(I - b / np.sum(b))))


def polish_gs(g: np.ndarray, G: np.ndarray, phase: np.ndarray, iters: int) -> np.ndarray:
    """iters Gerchberg-Saxton rounds (B3) from the given phase; returns the new phase."""
    g = np.asarray(g, dtype=np.float64)
    G = np.asarray(G, dtype=np.float64)
    W = dft_matrix(g.shape[0])
    Wc = np.conj(W)
    phi = np.asarray(phase, dtype=np.float64).copy()
    for _ in range(iters):
        F = W @ (g * np.exp(2j * np.pi * phi)) @ W.T
        mag = np.abs(F)
        unit = np.where(mag > 0, F / np.where(mag > 0, mag, 1.0), 1.0)
        f = Wc @ (G * unit) @ Wc.T
        phi = np.angle(f) / (2 * np.pi)
    return phi
