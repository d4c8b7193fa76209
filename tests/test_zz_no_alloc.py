"""fot_solve_noalloc (the entry point for callers that cannot allocate) against fot_solve.

Two calls in a row on the library's static scratch array, the second with a smaller grid and a
different operand type, each compared with a solve through an allocated plan (fot_plan +
fot_solve + fot_potentials) on the same inputs: the same kernels run in the same order, so
the potentials, phase and report values must be identical bit for bit."""
import sys

import numpy as np
import pytest

from paper_2512_19072_amd import workloads as W
from tests.parity_util import to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, B, seed):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 2, c - 1, 0.22 * n) + 0.02
    G = np.stack([np.sqrt(np.where(rng.uniform(0, 1, (n, n)) < 0.7, 1.0, 1e-6)) * W.gaussian(n, c, c, 0.3 * n)
                  for _ in range(B)])
    G[0, 4, :] = 0.0
    return g, G


def _with_plan(F, g, G, prec, eps, T):
    n, B = g.shape[0], G.shape[0]
    plan = F.Plan(n, B, prec, max_iters=T)
    ph, rep, st = plan.solve(to_dev(g), to_dev(G), eps, T, check=False)
    f, psi = plan.potentials()
    plan.close()
    return ph, f, psi, rep, st


def _noalloc(F, g, G, prec, eps, T):
    import torch
    n, B = g.shape[0], G.shape[0]
    dev = torch.device("cuda", 0)
    f = torch.full((B, n, n), 7.0, dtype=torch.float64, device=dev)
    psi = torch.full_like(f, 7.0)
    ph = torch.full_like(f, 7.0)
    rep = F.Report(B, T)
    st = F.fot_solve_noalloc(n, B, prec, to_dev(g), to_dev(G), eps, T, f_out=f, psi_out=psi, phase_out=ph,
                             report=rep.raw, check=False)
    return ph, f, psi, rep, st


@pytest.mark.parametrize("calls", [[(200, 2, "f32", 1e-2, 40), (96, 1, "bf16", 2e-2, 25)],
                                   # the largest FP32 grid the 32 MiB array holds for one target
                                   [(640, 1, "f32", 1e-2, 10), (128, 1, "f16", 5e-2, 10)],
                                   # and for FP64 operands
                                   [(640, 1, "f64", 1e-2, 10), (64, 1, "bf16x3", 2e-2, 10)]])
def test_noalloc_matches_allocated_plan(calls):
    import torch
    from paper_2512_19072_amd import fot as F
    for n, B, prec, eps, T in calls:
        _say(f"case: fot_solve_noalloc n={n} B={B} {prec} eps={eps} T={T}")
        g, G = _case(n, B, n)
        ph0, f0, psi0, rep0, st0 = _with_plan(F, g, G, prec, eps, T)
        ph1, f1, psi1, rep1, st1 = _noalloc(F, g, G, prec, eps, T)
        torch.cuda.synchronize()
        assert st0 == F.FOT_OK and st1 == F.FOT_OK, (st0, st1, F.fot_last_error())
        assert bool((f1 == f0).all()) and bool((psi1 == psi0).all()), "potentials differ"
        assert bool((ph1 == ph0).all()), "phase differs"
        for key in ("err_a", "err_b", "dual", "transport_cost", "err_products"):
            assert np.array_equal(getattr(rep1, key), getattr(rep0, key)), key
        assert np.array_equal(rep1.err_a_history, rep0.err_a_history)
        assert rep1.graph == 0 and rep1.ms_total == 0.0


def test_noalloc_rejects_what_it_cannot_hold():
    from paper_2512_19072_amd import fot as F
    import torch
    n = 1024                                   # the workspace of a 1024^2 plan exceeds 32 MiB
    g, G = _case(n, 1, 3)
    st = F.fot_solve_noalloc(n, 1, "f32", to_dev(g), to_dev(G), 1e-2, 5, check=False)
    assert st == F.FOT_E_INVALID and "scratch" in F.fot_last_error()
    with pytest.raises(F.FOTError):
        F.fot_solve_noalloc(64, 1, "f32", to_dev(g[:64, :64]), to_dev(G[:, :64, :64]), 1e-2, 5,
                            flags=F.FOT_FLAG_PROFILE)
    # still usable afterwards
    ph, f, psi, rep, st = _noalloc(F, *_case(64, 1, 4), "f64", 1e-2, 10)
    torch.cuda.synchronize()
    assert st == F.FOT_OK and bool(torch.isfinite(ph).all())
