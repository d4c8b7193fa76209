"""Pins of the output-beam and Gerchberg-Saxton oracle (oracle/beam.py) against what the
mathematics fixes: the transform's definition summed by brute force, an independent FFT route,
Parseval, the landing point of a linear phase (the sign convention), the beam of a solved
transport problem, and two textbook properties of Gerchberg-Saxton (a consistent phase is a
fixed point; the Fourier-plane error of error reduction never increases)."""
import math

import numpy as np
import pytest

import oracle as O
from oracle import beam as Bm


def _brute_field(g, phase):
    n = g.shape[0]
    c = n // 2
    F = np.zeros((n, n), dtype=np.complex128)
    for L in range(n):
        for M in range(n):
            s = 0j
            for j in range(n):
                for k in range(n):
                    arg = ((j - c) * (L - c) + (k - c) * (M - c)) / n
                    s += g[j, k] * np.exp(2j * math.pi * phase[j, k]) * np.exp(-2j * math.pi * arg)
            F[L, M] = s
    return F


@pytest.mark.parametrize("n", [5, 6])
def test_field_equals_brute_force_sum(n):
    rng = np.random.default_rng(n)
    g = rng.uniform(0, 1, (n, n))
    ph = rng.uniform(-1, 1, (n, n))
    F = Bm.output_field(g, ph)
    ref = _brute_field(g, ph)
    assert np.max(np.abs(F - ref)) < 1e-12 * np.max(np.abs(ref))


@pytest.mark.parametrize("n", [16, 17])
def test_field_equals_shifted_fft(n):
    rng = np.random.default_rng(100 + n)
    g = rng.uniform(0, 1, (n, n))
    ph = rng.uniform(-1, 1, (n, n))
    f = g * np.exp(2j * np.pi * ph)
    ref = np.fft.fftshift(np.fft.fft2(np.fft.ifftshift(f)))
    F = Bm.output_field(g, ph)
    assert np.max(np.abs(F - ref)) < 1e-11 * np.max(np.abs(ref))


def test_parseval_and_unit_power():
    n = 24
    rng = np.random.default_rng(7)
    g = rng.uniform(0, 1, (n, n))
    ph = rng.uniform(0, 1, (n, n))
    F = Bm.output_field(g, ph)
    assert abs(np.sum(np.abs(F) ** 2) - n * n * np.sum(g ** 2)) < 1e-10 * n * n * np.sum(g ** 2)
    I = Bm.output_beam(g, ph)
    assert abs(I.sum() - 1.0) < 1e-13
    assert np.max(np.abs(I - np.abs(F) ** 2 / (n * n * np.sum(g ** 2)))) < 1e-15


@pytest.mark.parametrize("n,a,b", [(16, 3, -2), (15, -4, 5)])
def test_linear_phase_lands_at_its_gradient(n, a, b):
    """phi = (a (j - c) + b (k - c)) / n has dphi/dx = a / sqrt(n) = X_{c+a}: a uniform beam lands
    entirely on pixel (c + a, c + b)."""
    c = n // 2
    j = np.arange(n)[:, None] - c
    k = np.arange(n)[None, :] - c
    ph = (a * j + b * k) / n
    I = Bm.output_beam(np.ones((n, n)), ph)
    assert abs(I[c + a, c + b] - 1.0) < 1e-12
    I[c + a, c + b] = 0.0
    assert np.max(I) < 1e-12


def test_solved_transport_phase_reaches_its_target():
    """The FOT phase of a Gaussian -> displaced Gaussian problem sends the beam onto the target:
    its L1 loss is far below that of a flat phase, and the output's centroid sits at the target's."""
    n = 32
    c = n // 2
    idx = np.arange(n) - c
    g = np.exp(-(idx[:, None] ** 2 + idx[None, :] ** 2) / (2 * 4.0 ** 2))
    G = np.exp(-((idx[:, None] - 5) ** 2 + (idx[None, :] + 3) ** 2) / (2 * 4.0 ** 2))
    res = O.solve_sep(g, G, 2e-3, 300)
    l_fot = Bm.l1_loss(g, res.phase, G)
    l_flat = Bm.l1_loss(g, np.zeros((n, n)), G)
    assert l_fot < 0.2 * l_flat, (l_fot, l_flat)
    I = Bm.output_beam(g, res.phase)
    cy = np.sum(I * idx[:, None])
    cx = np.sum(I * idx[None, :])
    assert abs(cy - 5) < 0.3 and abs(cx + 3) < 0.3, (cy, cx)


def test_consistent_phase_is_a_gs_fixed_point():
    n = 12
    rng = np.random.default_rng(3)
    g = rng.uniform(0.5, 1, (n, n))
    ph = rng.uniform(-0.5, 0.5, (n, n))
    G = np.abs(Bm.output_field(g, ph))
    out = Bm.polish_gs(g, G, ph, 3)
    d = np.abs(np.exp(2j * np.pi * out) - np.exp(2j * np.pi * ph))
    assert np.max(d) < 1e-10


def test_gs_fourier_error_never_increases():
    """Error reduction (Gerchberg-Saxton) with unit-power g and G: the Fourier-plane error
    sum (|F_k| / n - G)^2 of successive rounds is non-increasing."""
    n = 16
    rng = np.random.default_rng(11)
    g = rng.uniform(0, 1, (n, n))
    g /= np.sqrt(np.sum(g ** 2))
    G = rng.uniform(0, 1, (n, n)) * (rng.uniform(0, 1, (n, n)) < 0.5)
    G /= np.sqrt(np.sum(G ** 2))
    ph = rng.uniform(-0.5, 0.5, (n, n))
    errs = []
    for _ in range(12):
        F = Bm.output_field(g, ph)
        errs.append(float(np.sum((np.abs(F) / n - G) ** 2)))
        ph = Bm.polish_gs(g, G, ph, 1)
    assert all(e2 <= e1 * (1 + 1e-12) for e1, e2 in zip(errs, errs[1:])), errs
    assert errs[-1] < 0.9 * errs[0]


# planted mistakes: each must fail at least one of the pins above
_real_dft = Bm.dft_matrix


def _conj_dft(n):
    return np.conj(_real_dft(n))                                   # opposite sign convention


def _uncentred_dft(n):
    i = np.arange(n)
    return np.exp(-2j * np.pi * np.mod(np.outer(i, i), n) / n)      # forgot the centring


def _gs_without_conj(g, G, phase, iters):
    g = np.asarray(g, dtype=np.float64)
    W = _real_dft(g.shape[0])
    phi = np.asarray(phase, dtype=np.float64).copy()
    for _ in range(iters):
        F = W @ (g * np.exp(2j * np.pi * phi)) @ W.T
        mag = np.abs(F)
        f = W @ (G * F / np.where(mag > 0, mag, 1.0)) @ W.T          # forward transform as inverse
        phi = np.angle(f) / (2 * np.pi)
    return phi


@pytest.mark.parametrize("name,wrong,pins", [
    ("dft_matrix", _conj_dft, [lambda: test_linear_phase_lands_at_its_gradient(16, 3, -2)]),
    ("dft_matrix", _uncentred_dft, [lambda: test_field_equals_brute_force_sum(5)]),
    ("polish_gs", _gs_without_conj, [test_consistent_phase_is_a_gs_fixed_point]),
])
def test_planted_beam_mistakes_fail_a_pin(monkeypatch, name, wrong, pins):
    monkeypatch.setattr(Bm, name, wrong)
    failed = 0
    for pin in pins:
        try:
            pin()
        except AssertionError:
            failed += 1
    assert failed > 0, f"no pin caught the planted mistake in {name}"


def test_l1_loss_of_a_delta_beam():
    """A linear phase puts a uniform beam on one pixel: the loss against a target on that pixel is
    0 and against a target on another pixel 2 (two unit masses that do not overlap)."""
    n, a, b = 16, 2, 5
    c = n // 2
    j = np.arange(n)[:, None] - c
    k = np.arange(n)[None, :] - c
    ph = (a * j + b * k) / n
    G = np.zeros((n, n))
    G[c + a, c + b] = 3.0
    assert Bm.l1_loss(np.ones((n, n)), ph, G) < 1e-12
    G2 = np.zeros((n, n))
    G2[c - 1, c] = 1.0
    assert abs(Bm.l1_loss(np.ones((n, n)), ph, G2) - 2.0) < 1e-12
