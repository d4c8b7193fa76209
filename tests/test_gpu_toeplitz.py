"""The Toeplitz table of the Gibbs factor's operand against the same operand staged through LDS
with every K stage (FOT_FLAG_STAGED_LAMBDA).

Lambda[i][k] = exp(-(i - k)^2 / (2 n^2 eps)) depends on i - k only (Sec. 3, Eq. 7-8: the per-axis
kernel of the separable cost), so the fused kernels read its fragments from one table per
workgroup.  The table holds the very values of the stored Lambda and the MFMAs run in the same
order, so every result must be bit-identical to the staged form: potentials, phase, report
scalars and histories, and reverse-mode gradients.  The cases cover ragged sizes (padded rows
and columns), batches, both tile configurations, FP64 band skipping at small eps and every
operand type that uses the table."""
import sys

import numpy as np
import pytest

from paper_2512_19072_amd import workloads as W
from tests.parity_util import run_gpu, to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, B, seed):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 3, c - 2, 0.2 * n) + 0.05 * rng.uniform(0, 1, (n, n))
    g[-1, :] = 0.0
    Gs = []
    for b in range(B):
        G = np.sqrt(np.where(rng.uniform(0, 1, (n, n)) < 0.7, 1.0, 1e-6)) * W.gaussian(n, c + b, c, 0.35 * n)
        G[:, 0] = 0.0
        Gs.append(G)
    return g, np.stack(Gs)


def _same(a, b, what):
    assert a.shape == b.shape, what
    eq = (a == b) | (np.isnan(a) & np.isnan(b))
    assert eq.all(), f"{what}: {int((~eq).sum())} of {a.size} entries differ, max |diff| " \
                     f"{np.nanmax(np.abs(np.where(eq, 0.0, a - b)))}"


@pytest.mark.parametrize("n,B,prec,eps,T,small", [
    (72, 1, "f32", 2e-2, 30, False),
    (130, 2, "bf16", 2e-2, 30, False),
    (300, 1, "f16", 5e-2, 30, False),
    (200, 1, "f64", 1e-2, 30, False),
    (256, 1, "f64", 2e-4, 40, False),      # FP64 band skipping (Lambda's band narrower than n)
    (700, 1, "bf16", 1e-2, 20, True),      # 32 x 32 tiles on a grid that would take 64 x 64
    (1024, 1, "f32", 5e-3, 20, False),
    (1024, 1, "bf16", 5e-3, 20, False),
    # BF16x3: the hi and the lo halves from two tables
    (96, 2, "bf16x3", 2e-2, 30, False),
    (300, 1, "bf16x3", 1e-2, 30, False),
    (700, 1, "bf16x3", 1e-2, 20, True),
    (1024, 1, "bf16x3", 5e-3, 20, False),
])
def test_toeplitz_table_is_bit_identical_to_staged_lambda(n, B, prec, eps, T, small):
    g, Gs = _case(n, B, n)
    _say(f"case: toeplitz n={n} B={B} {prec} eps={eps} T={T} small_tiles={small}")
    a = run_gpu(g, Gs, eps, T, prec, small_tiles=small)
    b = run_gpu(g, Gs, eps, T, prec, small_tiles=small, staged_lambda=True)
    assert a["status"] == b["status"], (a["status"], b["status"])
    for k in ("f", "psi", "phase"):
        _same(a[k], b[k], k)
    ra, rb = a["rep"], b["rep"]
    for k in ("err_a", "err_b", "dual", "transport_cost", "err_a_history", "err_b_history"):
        _same(np.asarray(getattr(ra, k)), np.asarray(getattr(rb, k)), k)


@pytest.mark.parametrize("prec,f64_reverse", [("f32", False), ("f32", True), ("bf16", False)])
def test_toeplitz_table_reverse_mode_is_bit_identical(prec, f64_reverse):
    """Reverse half-steps (FP32 operands after an FP32 solve, FP64 otherwise) on the table and on
    staged Lambda: identical gradients."""
    from paper_2512_19072_amd import fot as F
    n, B, T, k, eps = 200, 2, 24, 5, 1e-2
    g, Gs = _case(n, B, 5)
    rng = np.random.default_rng(6)
    dD = np.array([0.6, -0.4])
    dphi = rng.standard_normal((B, n, n))
    _say(f"case: toeplitz reverse {prec} f64_reverse={f64_reverse}")
    out = []
    for staged in (False, True):
        plan = F.Plan(n, B, prec, max_iters=T, checkpoint_every=k, f64_reverse=f64_reverse, staged_lambda=staged)
        plan.solve(to_dev(g), to_dev(Gs), eps, T)
        out.append(plan.backward(dD, to_dev(dphi)).cpu().numpy())
    _same(out[0], out[1], "dL/dG")
