"""Helpers shared by the GPU parity tests: run the library, run the oracle, compare.

Comparison (the paper leaves potentials defined only up to (f + k, psi - k)): potentials are
gauge-fixed by subtracting their a- (resp. b-) weighted mean and compared on finite entries,
as max |x - ref| / (max ref - min ref); the phase likewise (it is defined up to a constant and
both sides remove the a-weighted mean); scalars relative to their magnitude.
"""
import numpy as np

import oracle as O


def device():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch.device("cuda", 0)


def to_dev(x):
    import torch
    return torch.tensor(np.ascontiguousarray(x), dtype=torch.float64, device=device())


def run_gpu(g, G, eps, iters, precision, checkpoint_every=0, max_iters=None, profile=False, **plan_kw):
    from paper_2512_19072_amd import fot as F
    G = np.asarray(G)
    if G.ndim == 2:
        G = G[None]
    n, B = g.shape[0], G.shape[0]
    plan = F.Plan(n, B, precision, max_iters=max_iters or iters, checkpoint_every=checkpoint_every,
                  profile=profile, **plan_kw)
    phase, rep, st = plan.solve(to_dev(g), to_dev(G), eps, iters)
    f, psi = plan.potentials()
    out = dict(phase=phase.cpu().numpy(), f=f.cpu().numpy(), psi=psi.cpu().numpy(), rep=rep, plan=plan,
               status=st)
    return out


def gauge_rel(x, ref, w):
    m = np.isfinite(ref)
    assert np.array_equal(np.isfinite(x), m), "different sets of infinite potentials"
    if not m.any():
        return 0.0
    xs = x[m] - np.sum(w[m] * x[m]) / np.sum(w[m])
    rs = ref[m] - np.sum(w[m] * ref[m]) / np.sum(w[m])
    rng = rs.max() - rs.min()
    return float(np.max(np.abs(xs - rs)) / (rng if rng > 0 else 1.0))


def range_rel(x, ref):
    rng = ref.max() - ref.min()
    return float(np.max(np.abs(x - ref)) / (rng if rng > 0 else 1.0))


def _hist_ratio(h, ref, rtol, floor):
    """max |h - ref| / (rtol ref + floor) over the finite entries; infinite entries must match."""
    fin = np.isfinite(ref)
    assert np.array_equal(np.isfinite(h), fin), "different sets of infinite marginal errors"
    if not fin.any():
        return 0.0
    return float(np.max(np.abs(h[fin] - ref[fin]) / (rtol * ref[fin] + floor)))


# Marginal errors shrink to the rounding floor of each precision, so they are compared as
# |gpu - ref| <= rtol * ref + floor; the entries report the worst ratio (pass if <= 1).
HIST_TOL = {"f64": (1e-6, 1e-12), "f32": (1e-3, 2e-6), "bf16": (0.1, 1e-3), "f16": (0.1, 1e-3),
            "bf16x3": (1e-2, 1e-5)}


def compare(gpu, ref, g, G, b_index=0, precision="f64"):
    """Dict of relative errors of one target of a GPU solve against an oracle Result."""
    a = O.normalise(g)
    b = O.normalise(G)
    rep = gpu["rep"]
    rtol, floor = HIST_TOL[precision]
    e = {}
    e["f"] = gauge_rel(gpu["f"][b_index], ref.f, a)
    e["psi"] = gauge_rel(gpu["psi"][b_index], ref.psi, b)
    e["phase"] = range_rel(gpu["phase"][b_index], ref.phase)
    e["dual"] = abs(rep.dual[b_index] - ref.dual) / max(abs(ref.dual), 1e-300)
    e["cost"] = abs(rep.transport_cost[b_index] - ref.cost) / max(abs(ref.cost), 1e-300)
    e["err_a"] = abs(rep.err_a[b_index] - ref.err_a) / (rtol * ref.err_a + floor)
    ha = rep.err_a_history[:, b_index]
    hb = rep.err_b_history[:, b_index]
    e["hist_a"] = _hist_ratio(ha, ref.err_a_hist, rtol, floor)
    e["hist_b"] = _hist_ratio(hb, ref.err_b_hist, rtol, floor)
    e["err_b_gpu"] = float(rep.err_b[b_index])
    e["err_a_values"] = (float(rep.err_a[b_index]), float(ref.err_a))
    return e


_WL1_REF = {}


def workload1_ref(g, G):
    """The oracle's solve of the 1024 x 1024 two-Gaussian workload (eps 5e-3, 200 iterations),
    computed once per test session and shared by the tests that compare against it."""
    if "ref" not in _WL1_REF:
        _WL1_REF["ref"] = O.solve_sep(g, G, 5e-3, 200)
    return _WL1_REF["ref"]
