"""CPU checks of the FFT-convolution reference (oracle/cfot.py): Eq. 11 holds to rounding while the
convolution values stay far above the FFT's rounding, and FP64 FFT convolution itself loses the
small values at small eps (the cFOT instability of Sec. 4), independently of the GPU."""
import numpy as np

import oracle as O
from oracle import cfot as C
from paper_2512_19072_amd import workloads as W


def _case(n, seed):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 2, c - 1, 0.2 * n) + 0.05 * rng.uniform(0, 1, (n, n))
    G = np.sqrt(np.where(rng.uniform(0, 1, (n, n)) < 0.7, 1.0, 1e-6)) * W.gaussian(n, c, c, 0.35 * n)
    G[:, 0] = 0.0
    G[3, :] = 0.0
    return g, G


def test_conv_rows_equals_direct_product():
    n, eps = 37, 2e-2
    rng = np.random.default_rng(1)
    L = rng.normal(0, 3, (5, n))
    L[2] = -np.inf                     # a row without mass
    L[3, :10] = -np.inf
    N = C.fft_length(n)
    got = C.conv_log_rows(L, C.lambda_transform(n, N, eps))
    lam = O.gibbs_1d(n, eps)
    with np.errstate(divide="ignore"):
        ref = np.log(np.exp(L) @ lam)
    assert np.array_equal(np.isfinite(got), np.isfinite(ref))
    fin = np.isfinite(ref)
    assert np.max(np.abs(got[fin] - ref[fin])) < 1e-12
    assert np.all(got[2] == -np.inf)


def test_convolution_solve_equals_matrix_products():
    n, T = 40, 30
    g, G = _case(n, 2)
    for eps in (2e-2, W.anneal_schedule(5e-2, 1e-2, T)):
        f, psi = C.solve_conv(g, G, eps, T)
        ref = O.solve_sep(g, G, eps, T)
        for x, r in ((f, ref.f), (psi, ref.psi)):
            m = np.isfinite(r)
            assert np.array_equal(np.isfinite(x), m)
            assert np.max(np.abs(x[m] - r[m])) < 1e-12 * np.ptp(r[m]) + 1e-14


def test_fft_convolution_loses_small_values_at_small_eps():
    """Two-Gaussian -> shapes at 128^2: FP64 FFT convolution stays finite at eps = 5e-3 and produces
    non-finite potentials within 100 iterations at eps = 2e-3, where the matrix products do not."""
    n, T = 128, 100
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    a, b = O.normalise(g), O.normalise(G)
    f, psi = C.solve_conv(g, G, 5e-3, T)
    assert np.all(np.isfinite(f[a > 0])) and np.all(np.isfinite(psi[b > 0]))
    with np.errstate(all="ignore"):
        f2, psi2 = C.solve_conv(g, G, 2e-3, T)
    assert not (np.all(np.isfinite(f2[a > 0])) and np.all(np.isfinite(psi2[b > 0])))
    ref = O.solve_sep(g, G, 2e-3, T)
    assert np.all(np.isfinite(ref.f[a > 0])) and np.all(np.isfinite(ref.psi[b > 0]))
