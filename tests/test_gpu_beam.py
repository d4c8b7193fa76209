"""GPU parity of the output beam (fot_output_beam) and Gerchberg-Saxton polishing
(fot_polish_gs) against the FP64 oracle in oracle/beam.py, through the C ABI.

Both sides compute in FP64 (the GPU's transform is four FP64 MFMA GEMMs, the oracle's two
complex matrix products), so intensities and losses agree to ~1e-13 relative; the tests use
1e-11.  Phases after Gerchberg-Saxton are compared as unit phasors e^{2 pi i phi} on pixels that
carry light (a phase is defined modulo 1)."""
import sys

import numpy as np
import pytest

import oracle as O
from oracle import beam as Bm
from paper_2512_19072_amd import workloads as W
from tests.parity_util import to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, seed, B=1):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 1, c - 2, 0.25 * n) + 0.02 * rng.uniform(0, 1, (n, n))
    g[0, :] = 0.0
    G = np.stack([W.gaussian(n, c + 3 * b, c - 4, 0.2 * n) * (rng.uniform(0, 1, (n, n)) < 0.8) for b in range(B)])
    ph = rng.uniform(-0.5, 0.5, (B, n, n))
    return g, G, ph


def _phasor_err(a, b, w):
    m = w > 1e-3 * w.max()
    return float(np.max(np.abs(np.exp(2j * np.pi * a[m]) - np.exp(2j * np.pi * b[m]))))


@pytest.mark.parametrize("n,B", [(72, 2), (130, 1), (1, 1), (3, 1)])
def test_output_beam_matches_oracle(n, B):
    from paper_2512_19072_amd import fot as F
    g, G, ph = _case(n, n, B)
    if n <= 3:
        g = np.arange(1, n * n + 1, dtype=np.float64).reshape(n, n)
        G = np.arange(n * n, 0, -1, dtype=np.float64).reshape(1, n, n)
    _say(f"case: output beam n={n} B={B}")
    plan = F.Plan(n, B, "f64", max_iters=1)
    I, l1 = plan.output_beam(to_dev(g), to_dev(ph), to_dev(G))
    I = I.cpu().numpy()
    plan.close()
    for b in range(B):
        ref_I = Bm.output_beam(g, ph[b])
        ref_l1 = Bm.l1_loss(g, ph[b], G[b])
        e_I = np.max(np.abs(I[b] - ref_I)) / np.max(ref_I)
        e_l = abs(l1[b] - ref_l1) / max(ref_l1, 1.0)   # (n = 1: the loss is exactly 0)
        _say(f"  target {b}: intensity {e_I:.2e}, l1 {e_l:.2e} (l1 = {ref_l1:.4f})")
        assert e_I < 1e-11 and e_l < 1e-11


def test_linear_phase_lands_at_its_gradient():
    from paper_2512_19072_amd import fot as F
    n, a, b = 96, 7, -5
    c = n // 2
    j = np.arange(n)[:, None] - c
    k = np.arange(n)[None, :] - c
    ph = ((a * j + b * k) / n)[None]
    plan = F.Plan(n, 1, "f32", max_iters=1)
    I, l1 = plan.output_beam(to_dev(np.ones((n, n))), to_dev(ph), intensity=True)
    plan.close()
    I = I.cpu().numpy()[0]
    assert l1 is None
    assert abs(I[c + a, c + b] - 1.0) < 1e-12
    I[c + a, c + b] = 0.0
    assert np.max(I) < 1e-12


@pytest.mark.parametrize("n", [64, 100])
def test_gs_matches_oracle(n):
    from paper_2512_19072_amd import fot as F
    g, G, ph = _case(n, 50 + n)
    _say(f"case: GS n={n} 5 rounds")
    plan = F.Plan(n, 1, "f32", max_iters=1)
    phd = to_dev(ph)
    plan.polish_gs(to_dev(g), to_dev(G), phd, 5)
    got = phd.cpu().numpy()[0]
    ref = Bm.polish_gs(g, G[0], ph[0], 5)
    e = _phasor_err(got, ref, g)
    _say(f"  phasor error {e:.2e}")
    assert e < 1e-9
    assert np.all(got > -0.5 - 1e-15) and np.all(got <= 0.5 + 1e-15)
    phz = to_dev(ph)
    plan.polish_gs(to_dev(g), to_dev(G), phz, 0)
    assert bool((phz.cpu() == to_dev(ph).cpu()).all())
    plan.close()


def test_fot_then_gs_lowers_the_loss():
    """The FOT phase of a solved problem beats a flat phase by far, and Gerchberg-Saxton rounds
    started from it lower the L1 intensity loss further (the paper's pipeline, Sec. 4)."""
    from paper_2512_19072_amd import fot as F
    n = 128
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 3 else G[None]
    gd, Gd = to_dev(g), to_dev(G)
    _say(f"case: FOT + GS n={n}")
    plan = F.Plan(n, 1, "f32", max_iters=200)
    ph, rep, _ = plan.solve(gd, Gd, 5e-3, 200)
    _, l_fot = plan.output_beam(gd, ph, Gd, intensity=False)
    _, l_flat = plan.output_beam(gd, to_dev(np.zeros((1, n, n))), Gd, intensity=False)
    ref = Bm.l1_loss(g, ph.cpu().numpy()[0], G[0])
    plan.polish_gs(gd, Gd, ph, 20)
    _, l_gs = plan.output_beam(gd, ph, Gd, intensity=False)
    plan.close()
    _say(f"  L1: flat {l_flat[0]:.4f}, FOT {l_fot[0]:.4f} (oracle {ref:.4f}), FOT + 20 GS {l_gs[0]:.4f}")
    assert abs(l_fot[0] - ref) < 1e-11 * ref
    assert l_fot[0] < 0.5 * l_flat[0]
    assert l_gs[0] < l_fot[0]


def test_invalid_beam_inputs():
    from paper_2512_19072_amd import fot as F
    n = 64
    g, G, ph = _case(n, 9)
    plan = F.Plan(n, 1, "f32", max_iters=1)
    bad = g.copy()
    bad[3, 3] = -1.0
    with pytest.raises(F.FOTError) as e:
        plan.output_beam(to_dev(bad), to_dev(ph), to_dev(G))
    assert e.value.status == F.FOT_E_INVALID
    with pytest.raises(F.FOTError):
        F.fot_output_beam(plan.handle, to_dev(g), to_dev(ph), None, None, np.zeros(1))
    with pytest.raises(F.FOTError):
        plan.polish_gs(to_dev(g), to_dev(G), to_dev(ph), -1)
    with pytest.raises(F.FOTError):
        plan.output_beam(to_dev(g), to_dev(ph), to_dev(np.zeros((1, n, n))))
    # the plan stays usable
    I, l1 = plan.output_beam(to_dev(g), to_dev(ph), to_dev(G))
    assert abs(l1[0] - Bm.l1_loss(g, ph[0], G[0])) < 1e-11
    plan.close()


def test_workload1_full_size_beam_and_gs():
    """1024^2: the output beam and loss of the FP32 FOT phase, and two GS rounds, against the
    oracle.  Over 1024^2-term FP64 sums the two sides' rounding differs by ~1e-13 of the field's
    scale; a GS phase is the argument of the back-transformed field, so where that field is small
    the difference grows in proportion (1.6e-8 measured): the bound is 1e-7 here."""
    from paper_2512_19072_amd import fot as F
    wl = W.workload(1)
    g, G = wl.images()
    n = wl.n
    gd, Gd = to_dev(g), to_dev(G)
    _say("case: twogauss_to_shapes n=1024 beam + 2 GS rounds")
    plan = F.Plan(n, 1, "f32", max_iters=200)
    ph, _, _ = plan.solve(gd, Gd, 5e-3, 200)
    I, l1 = plan.output_beam(gd, ph, Gd)
    ph0 = ph.cpu().numpy()[0]
    plan.polish_gs(gd, Gd, ph, 2)
    got = ph.cpu().numpy()[0]
    I = I.cpu().numpy()[0]
    plan.close()
    _say("  gpu done; oracle running")
    ref_I = Bm.output_beam(g, ph0)
    ref_l1 = Bm.l1_loss(g, ph0, G[0])
    e_I = np.max(np.abs(I - ref_I)) / np.max(ref_I)
    _say(f"  intensity {e_I:.2e}, l1 {l1[0]:.5f} vs {ref_l1:.5f}")
    assert e_I < 1e-11 and abs(l1[0] - ref_l1) < 1e-11 * ref_l1
    ref = Bm.polish_gs(g, G[0], ph0, 2)
    e = _phasor_err(got, ref, g)
    _say(f"  GS phasor error {e:.2e}")
    assert e < 1e-7
