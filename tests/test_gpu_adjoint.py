"""GPU reverse mode (fot_backward through the C ABI) against the oracle's reverse sweep and
against central finite differences.

Tolerances: FP64 operands 1e-9 of the gradient's max magnitude against the oracle (both are
FP64; they differ in summation order only); FP32 operands (forward, and reverse half-steps unless
FOT_FLAG_F64_REVERSE) 1e-4 against FP64 finite differences and the oracle (the stated target)."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_2512_19072_amd import workloads as W
from tests.parity_util import to_dev

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _case(n, B, seed, zero=True):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 1, c - 2, 0.25 * n) + 0.05
    Gs = np.stack([np.sqrt(np.where(rng.uniform(0, 1, (n, n)) < 0.6, 1.0, 1e-3)) * W.gaussian(n, c, c, 0.4 * n)
                   for _ in range(B)])
    if zero:
        Gs[0, 2, 3] = 0.0
    return g, Gs


def _gpu_grad(g, Gs, eps, T, k, prec, dD, dphi, f64_reverse=False):
    import torch
    from paper_2512_19072_amd import fot as F
    n, B = g.shape[0], Gs.shape[0]
    plan = F.Plan(n, B, prec, max_iters=T, checkpoint_every=k, f64_reverse=f64_reverse)
    plan.solve(to_dev(g), to_dev(Gs), eps, T)
    dG = plan.backward(dD, None if dphi is None else to_dev(dphi))
    return dG.cpu().numpy()


@pytest.mark.parametrize("with_phase", [False, True])
def test_backward_matches_oracle_f64(with_phase):
    n, B, T, k, eps = 24, 2, 12, 5, 3e-2
    g, Gs = _case(n, B, 1)
    rng = np.random.default_rng(2)
    dD = np.array([0.7, -0.3])
    dphi = rng.standard_normal((B, n, n)) if with_phase else None
    _say(f"case: backward f64 n={n} B={B} T={T} k={k} phase={with_phase}")
    got = _gpu_grad(g, Gs, eps, T, k, "f64", dD, dphi)
    for b in range(B):
        ref = O.grad_G(g, Gs[b], eps, T, dD[b], None if dphi is None else dphi[b])
        err = np.max(np.abs(got[b] - ref)) / np.max(np.abs(ref))
        _say(f"target {b}: rel err {err:.2e}")
        assert err < 1e-9, (b, err)
    assert got[0, 2, 3] == 0.0


def test_backward_f32_forward_block_normalised_lambda():
    """FP32 forward at an eps where Lambda is stored block-normalised (n = 64, eps = 2e-3: Lambda's
    raw FP32 band is 43 px), FP64 reverse sweep, against the oracle's FP64 gradient: within the
    FP32 target of 1e-4 of the gradient's largest magnitude."""
    n, B, T, k, eps = 64, 1, 12, 4, 2e-3
    g, Gs = _case(n, B, 7, zero=False)
    rng = np.random.default_rng(8)
    dphi = rng.standard_normal((B, n, n))
    _say(f"case: backward f32 forward n={n} eps={eps} T={T} k={k}")
    got = _gpu_grad(g, Gs, eps, T, k, "f32", [0.9], dphi)
    ref = O.grad_G(g, Gs[0], eps, T, 0.9, dphi[0])
    err = np.max(np.abs(got[0] - ref)) / np.max(np.abs(ref))
    _say(f"rel err {err:.2e}")
    assert err < 1e-4, err


@pytest.mark.parametrize("f64_reverse", [False, True])
def test_backward_f32_forward_raw_lambda(f64_reverse):
    """FP32 forward with Lambda held raw (n = 64, eps = 2e-2): the reverse half-steps run with FP32
    operands (the default) or FP64 ones (FOT_FLAG_F64_REVERSE); both within the FP32 target of 1e-4
    of the oracle's FP64 gradient, the FP64 reverse closer."""
    n, B, T, k, eps = 64, 2, 16, 5, 2e-2
    g, Gs = _case(n, B, 9)
    rng = np.random.default_rng(10)
    dphi = rng.standard_normal((B, n, n))
    dD = [0.8, -0.4]
    _say(f"case: backward f32 forward raw Lambda n={n} T={T} k={k} f64_reverse={f64_reverse}")
    got = _gpu_grad(g, Gs, eps, T, k, "f32", dD, dphi, f64_reverse=f64_reverse)
    for b in range(B):
        ref = O.grad_G(g, Gs[b], eps, T, dD[b], dphi[b])
        err = np.max(np.abs(got[b] - ref)) / np.max(np.abs(ref))
        _say(f"target {b}: rel err {err:.2e}")
        assert err < 1e-4, (b, err)
    assert got[0, 2, 3] == 0.0


def test_backward_f32_forward_mixed_reverse_types():
    """An annealed FP32 solve whose eps crosses from raw Lambda (FP32 reverse half-steps) to the
    block-normalised form (FP64 reverse half-steps): a reverse half-step hands its successor a
    ready operand only within one type, and the gradient stays within 1e-4 of the oracle's."""
    n, B, T, k = 64, 1, 14, 4
    e = W.anneal_schedule(2e-2, 2e-3, T)
    g, Gs = _case(n, B, 11, zero=False)
    rng = np.random.default_rng(12)
    dphi = rng.standard_normal((B, n, n))
    _say(f"case: backward f32 forward annealed n={n} T={T} k={k}")
    got = _gpu_grad(g, Gs, e, T, k, "f32", [1.1], dphi)
    ref = O.grad_G(g, Gs[0], e, T, 1.1, dphi[0])
    err = np.max(np.abs(got[0] - ref)) / np.max(np.abs(ref))
    _say(f"rel err {err:.2e}")
    assert err < 1e-4, err


def test_backward_annealed_f64():
    n, B, T, k = 20, 1, 9, 4
    g, Gs = _case(n, B, 3, zero=False)
    e = W.anneal_schedule(6e-2, 1e-2, T)
    rng = np.random.default_rng(4)
    dphi = rng.standard_normal((B, n, n))
    got = _gpu_grad(g, Gs, e, T, k, "f64", [1.3], dphi)
    ref = O.grad_G(g, Gs[0], e, T, 1.3, dphi[0])
    assert np.max(np.abs(got[0] - ref)) / np.max(np.abs(ref)) < 1e-9


@pytest.mark.parametrize("prec,eps", [("f32", 2e-2), ("bf16x3", 2e-2), ("f32", 2e-3), ("f64", 2e-2)])
def test_checkpoint_interval_is_bit_invariant(prec, eps):
    """The replayed segments reproduce the forward iterations bit for bit whatever the operand
    type, so the gradient does not depend on the checkpoint interval (at eps = 2e-3 the FP32
    operands use the block-normalised Gibbs factor, in the forward solve and in the replays; FP64
    needs the operand's exp(x - K ln 2) as an explicit FMA, which the compiler would otherwise
    contract differently in the prep kernel and in the pass-2 epilogue)."""
    n, B, T = 40, 2, 12
    g, Gs = _case(n, B, 5)
    rng = np.random.default_rng(6)
    dphi = rng.standard_normal((B, n, n))
    outs = [_gpu_grad(g, Gs, eps, T, k, prec, [1.0, 0.5], dphi) for k in (1, 5, 12)]
    assert np.array_equal(outs[0], outs[1]) and np.array_equal(outs[0], outs[2])


@pytest.mark.parametrize("prec", ["f32", "f64"])
def test_backward_twice_is_identical(prec):
    """The forward solve leaves its last checkpoint segment's iterates in the segment buffers, and
    the first backward pass uses them instead of replaying that segment; it then replays the others
    into the same buffers, so a second backward pass on the same tape must replay the last segment
    too. Both give the same bits."""
    import torch
    from paper_2512_19072_amd import fot as F
    n, B, T, k, eps = 48, 2, 12, 5, 2e-2
    g, Gs = _case(n, B, 13)
    rng = np.random.default_rng(14)
    dphi = to_dev(rng.standard_normal((B, n, n)))
    plan = F.Plan(n, B, prec, max_iters=T, checkpoint_every=k)
    plan.solve(to_dev(g), to_dev(Gs), eps, T)
    d1 = plan.backward([0.5, 1.0], dphi).cpu().numpy()
    d2 = plan.backward([0.5, 1.0], dphi).cpu().numpy()
    plan.close()
    assert np.all(np.isfinite(d1)) and np.array_equal(d1, d2)


def test_backward_requires_tape():
    from paper_2512_19072_amd import fot as F
    n = 32
    g, Gs = _case(n, 1, 7)
    plan = F.Plan(n, 1, "f32", max_iters=4, checkpoint_every=0)
    plan.solve(to_dev(g), to_dev(Gs), 1e-2, 4)
    with pytest.raises(F.FOTError) as ei:
        plan.backward([1.0], None)
    assert ei.value.status == F.FOT_E_STATE
    plan2 = F.Plan(n, 1, "f32", max_iters=4, checkpoint_every=2)
    with pytest.raises(F.FOTError) as ei:
        plan2.backward([1.0], None)
    assert ei.value.status == F.FOT_E_STATE


def _loss_batch(plan, gd, Gpert, eps, T, dD, dphi):
    """Per-target dD * D + <dphi, phase> for a batch of perturbed targets."""
    ph, rep, _ = plan.solve(gd, to_dev(Gpert), eps, T)
    ph = ph.cpu().numpy()
    return rep.dual * dD + np.einsum("bij,bij->b", ph, dphi)


def test_backward_matches_fd_f64():
    """GPU FP64 adjoint against central differences of GPU FP64 solves (batched perturbations)."""
    from paper_2512_19072_amd import fot as F
    n, T, eps, h = 48, 25, 2e-2, 1e-5
    g, Gs = _case(n, 1, 8, zero=False)
    rng = np.random.default_rng(9)
    dphi = rng.standard_normal((n, n))
    dD = 0.8
    grad = _gpu_grad(g, Gs, eps, T, 7, "f64", [dD], dphi[None])[0]
    pix = rng.choice(n * n, size=12, replace=False)
    Gp = np.repeat(Gs, 2 * len(pix), axis=0)
    for i, q in enumerate(pix):
        Gp[2 * i].flat[q] += h
        Gp[2 * i + 1].flat[q] -= h
    plan = F.Plan(n, Gp.shape[0], "f64", max_iters=T)
    L = _loss_batch(plan, to_dev(g), Gp, eps, T, dD, np.repeat(dphi[None], Gp.shape[0], axis=0))
    fd = (L[0::2] - L[1::2]) / (2 * h)
    adj = grad.flat[pix]
    err = np.max(np.abs(adj - fd)) / np.max(np.abs(fd))
    _say(f"fd f64: rel err {err:.2e}")
    assert err < 1e-6


def test_autograd_function_matches_backward():
    import torch
    from paper_2512_19072_amd import fot as F
    n, T, eps = 32, 10, 2e-2
    g, Gs = _case(n, 2, 10)
    gd = to_dev(g)
    Gd = to_dev(Gs).requires_grad_(True)
    plan = F.Plan(n, 2, "f64", max_iters=T, checkpoint_every=4)
    dual, phase = F.fot_apply(Gd, gd, plan, eps, T)
    a = torch.tensor(O.normalise(g), device=gd.device)
    loss = dual.sum() + 0.5 * (a * phase * phase).sum()
    loss.backward()
    ref = np.stack([O.grad_G(g, Gs[b], eps, T, 1.0, O.normalise(g) * phase[b].detach().cpu().numpy())
                    for b in range(2)])
    got = Gd.grad.cpu().numpy()
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-9


def test_autograd_stale_tape_raises():
    """Two differentiable solves on one plan: the plan's tape belongs to the second, so the
    backward of the first must raise instead of returning the second's gradient."""
    import torch
    from paper_2512_19072_amd import fot as F
    n, T, eps = 32, 6, 2e-2
    g, Gs = _case(n, 1, 11)
    gd = to_dev(g)
    G1 = to_dev(Gs).requires_grad_(True)
    G2 = to_dev(Gs * 0.9 + 0.05).requires_grad_(True)
    plan = F.Plan(n, 1, "f64", max_iters=T, checkpoint_every=3)
    d1, _ = F.fot_apply(G1, gd, plan, eps, T)
    d2, _ = F.fot_apply(G2, gd, plan, eps, T)
    d2.sum().backward()                     # the latest solve: fine
    assert G2.grad is not None and torch.all(torch.isfinite(G2.grad))
    with pytest.raises(RuntimeError, match="tape no longer belongs"):
        d1.sum().backward()
    plan.close()


def test_workload4_full_size_adjoint():
    """512 x 512, 8 targets, FP32 operands, 100 iterations, checkpoints every 10.
    L = D + 1/2 sum_p a_p (phi_p - phi0_p)^2 with phi0 = 0 per target.  Checked against
    central differences (h = 1e-4 on G, FP64 solves) on 64 pixels of each of the 8 targets,
    and against the oracle's gradient of target 0."""
    import torch
    from paper_2512_19072_amd import fot as F
    wl = W.workload(4)
    g, Gs = wl.images()
    n, B, T, eps, h = wl.n, wl.batch, wl.iters, float(wl.eps[0]), 1e-4
    a = O.normalise(g)
    gd = to_dev(g)
    _say("case: gauss_to_ellipses 512 B=8 f32 adjoint")
    plan = F.Plan(n, B, "f32", max_iters=T, checkpoint_every=wl.checkpoint_every)
    ph, rep, _ = plan.solve(gd, to_dev(Gs), eps, T)
    dphi = (torch.tensor(a, device=gd.device)[None] * ph).contiguous()
    dG = plan.backward(np.ones(B), dphi).cpu().numpy()
    assert np.all(np.isfinite(dG))
    plan.close()
    for b in range(B):
        pix = W.fd_pixels(n, b, 64)
        Gp = np.repeat(Gs[b:b + 1], 2 * len(pix), axis=0)
        for i, q in enumerate(pix):
            Gp[2 * i].flat[q] += h
            Gp[2 * i + 1].flat[q] -= h
        fplan = F.Plan(n, Gp.shape[0], "f64", max_iters=T)
        php, repp, _ = fplan.solve(gd, to_dev(Gp), eps, T)
        php = php.cpu().numpy()
        Lp = repp.dual + 0.5 * np.einsum("ij,bij->b", a, php * php)
        fplan.close()
        fd = (Lp[0::2] - Lp[1::2]) / (2 * h)
        adj = dG[b].flat[pix]
        err = np.max(np.abs(adj - fd)) / np.max(np.abs(fd))
        _say(f"target {b}: adjoint vs FD rel err {err:.2e}")
        assert err < 1e-4, (b, err)
    ref = O.grad_G(g, Gs[0], eps, T, 1.0, a * O.solve_sep(g, Gs[0], eps, T).phase)
    err0 = np.max(np.abs(dG[0] - ref)) / np.max(np.abs(ref))
    _say(f"target 0: adjoint vs oracle gradient rel err {err0:.2e}")
    assert err0 < 1e-4
