"""GPU parity of the HIP path (through the C ABI) against the FP64 oracle.

Tolerances (range-normalised, gauge-fixed; see tests/parity_util.py):
  FP64 operands  1e-10: FP64 MFMA and FP64 BLAS differ only in summation order; after 200
                 iterations of a contractive map the differences stay ~1e-13.
  FP32 operands  1e-6 on potentials and phase (the stated target); scalars 1e-6.
  BF16 operands  1e-3 on potentials (the stated target).
  BF16x3         1e-5: hi + lo holds a value to about 2^-17 and the dropped lo.lo term is
                 below 2^-16 of a product, so one contraction is accurate to ~1e-5 relative
                 in the worst case and to ~1e-7 on average over the sums.
"""
import math
import sys

import numpy as np
import pytest

import oracle as O
from paper_2512_19072_amd import workloads as W
from tests.parity_util import compare, run_gpu, workload1_ref

pytestmark = pytest.mark.gpu


def _say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def _rand_case(n, seed, zeros=True):
    rng = np.random.default_rng(seed)
    c = n // 2
    g = W.gaussian(n, c + 3, c - 2, 0.2 * n) + 0.05 * rng.uniform(0, 1, (n, n))
    G = np.sqrt(np.where(rng.uniform(0, 1, (n, n)) < 0.7, 1.0, 1e-6)) * W.gaussian(n, c, c, 0.35 * n)
    if zeros:
        G[:, 0] = 0.0
        G[3, :] = 0.0
        g[-1, :] = 0.0
    return g, G


def test_workload0_f64_matches_oracle():
    """64 x 64 Gaussian -> hard disk (exact zeros), FP64, 200 iterations."""
    wl = W.workload(0)
    g, G = wl.images()
    _say("case: gauss_to_disk n=64 f64 200 it")
    gpu = run_gpu(g, G, 1e-2, 200, "f64")
    ref = O.solve_sep(g, G[0], 1e-2, 200)
    e = compare(gpu, ref, g, G[0], precision="f64")
    _say(e)
    for k in ("f", "psi", "phase", "dual", "cost"):
        assert e[k] < 1e-10, (k, e[k])
    assert e["err_a"] <= 1 and e["hist_a"] <= 1 and e["hist_b"] <= 1, e
    assert e["err_b_gpu"] < 1e-13
    assert gpu["rep"].nonfinite == 0


@pytest.mark.parametrize("n,prec", [(100, "f64"), (100, "f32"), (130, "f32"), (72, "bf16"), (72, "f16"),
                                    (72, "bf16x3"), (130, "bf16x3")])
def test_ragged_sizes(n, prec):
    """Sizes that are not multiples of the 64-pixel tile, with zero rows/columns."""
    g, G = _rand_case(n, n)
    eps, T = 2e-2, 60
    _say(f"case: ragged n={n} {prec}")
    gpu = run_gpu(g, G, eps, T, prec)
    ref = O.solve_sep(g, G, eps, T)
    e = compare(gpu, ref, g, G, precision=prec)
    _say(e)
    tol = {"f64": 1e-10, "f32": 1e-6, "bf16": 1e-3, "f16": 1e-3, "bf16x3": 1e-5}[prec]
    for k in ("f", "psi", "phase"):
        assert e[k] < tol, (k, e[k])
    assert e["dual"] < tol
    assert e["hist_a"] <= 1 and e["hist_b"] <= 1, e


def test_batch_targets_are_independent():
    n, B, eps, T = 96, 3, 1e-2, 40
    rng = np.random.default_rng(3)
    g = W.gaussian(n, n // 2, n // 2, 20.0)
    Gs = np.stack([_rand_case(n, 10 + b)[1] for b in range(B)])
    _say(f"case: batch n={n} B={B} f32")
    gpu = run_gpu(g, Gs, eps, T, "f32")
    for b in range(B):
        ref = O.solve_sep(g, Gs[b], eps, T)
        e = compare(gpu, ref, g, Gs[b], b_index=b, precision="f32")
        assert e["f"] < 1e-6 and e["psi"] < 1e-6 and e["phase"] < 1e-6, (b, e)


@pytest.mark.parametrize("prec", ["f32", "bf16"])
def test_small_and_large_tile_configurations_agree(prec):
    """The fused kernels run on 32 x 32 tiles when 64 x 64 tiles would occupy at most half of the
    CUs (one 512^2 target: 64 tiles) and on 64 x 64 tiles otherwise (four 512^2 targets: 256
    tiles).  The same target solved both ways agrees with the oracle to the precision's
    tolerance."""
    import torch
    n, eps, T = 512, 1e-2, 40
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if not (128 <= cus < 512):
        pytest.skip(f"{cus} CUs: both 512^2 cases would use the same tile size")
    g, G = _rand_case(n, 21)
    _say(f"case: tile configurations n={n} {prec} B=1 and B=4")
    one = run_gpu(g, G, eps, T, prec)
    four = run_gpu(g, np.stack([G] * 4), eps, T, prec)
    ref = O.solve_sep(g, G, eps, T)
    tol = {"f32": 1e-6, "bf16": 1e-3}[prec]
    e1 = compare(one, ref, g, G, precision=prec)
    _say(e1)
    for k in ("f", "psi", "phase"):
        assert e1[k] < tol, (k, e1[k])
    for b in range(4):
        e4 = compare(four, ref, g, G, b_index=b, precision=prec)
        for k in ("f", "psi", "phase"):
            assert e4[k] < tol, (b, k, e4[k])
    # the batch entries are bit-identical to each other (one code path, independent targets)
    assert all(np.array_equal(four["psi"][0], four["psi"][b]) for b in range(1, 4))


@pytest.mark.parametrize("n,prec", [(600, "f32"), (700, "f32"), (700, "bf16")])
def test_ragged_sizes_around_the_tile_threshold(n, prec):
    """Ragged sizes on both sides of the tile-size choice: 600^2 pads to 640 (100 tiles of 64 x 64,
    under half of the CUs: 32 x 32 tiles), 700^2 to 768 (144 tiles: 64 x 64).  Two-Gaussian
    workload, eps 5e-3, against the oracle."""
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    T = 40
    _say(f"case: ragged around the tile threshold n={n} {prec}")
    gpu = run_gpu(g, G, 5e-3, T, prec)
    ref = O.solve_sep(g, G, 5e-3, T)
    e = compare(gpu, ref, g, G, precision=prec)
    _say({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()})
    tol = {"f32": 1e-6, "bf16": 1e-3}[prec]
    for k in ("f", "psi", "phase"):
        assert e[k] < tol, (k, e[k])
    assert e["dual"] < tol


def test_batch_at_the_papers_eps():
    """Two targets at eps = 2e-4 on 512^2 in FP32: small-grid tiles, the block-normalised Gibbs
    factor (shared by the batch) and per-target operands together, each against the oracle."""
    n, T, eps = 512, 40, 2e-4
    g, G1 = W.twogauss_to_shapes(n)
    G1 = G1 if G1.ndim == 2 else G1[0]
    G2 = np.ascontiguousarray(G1[::-1, :])
    Gs = np.stack([G1, G2])
    _say("case: batch of 2 at eps 2e-4, n=512 f32")
    gpu = run_gpu(g, Gs, eps, T, "f32")
    for b in range(2):
        ref = O.solve_sep(g, Gs[b], eps, T)
        e = compare(gpu, ref, g, Gs[b], b_index=b, precision="f32")
        _say(b, {k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()})
        assert e["f"] < 1e-6 and e["psi"] < 1e-6 and e["phase"] < 1e-6, (b, e)


def test_deterministic_and_warm_start():
    """Two solves are bit-identical; 30 + 30 warm-started iterations equal 60 iterations."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n = 128
    g, G = _rand_case(n, 5)
    gd, Gd = to_dev(g), to_dev(G[None])
    plan = F.Plan(n, 1, "f32", max_iters=60)
    p1, r1, _ = plan.solve(gd, Gd, 1e-2, 60)
    f1, s1 = plan.potentials()
    p2, r2, _ = plan.solve(gd, Gd, 1e-2, 60)
    f2, s2 = plan.potentials()
    assert bool((p1 == p2).all()) and bool((f1 == f2).all()) and bool((s1 == s2).all())
    assert np.array_equal(r1.err_a_history, r2.err_a_history) and r1.dual[0] == r2.dual[0]
    plan.solve(gd, Gd, 1e-2, 30)
    p3, r3, _ = plan.solve(gd, Gd, 1e-2, 30, warm_start=True)
    f3, s3 = plan.potentials()
    assert bool((f3 == f1).all()) and bool((s3 == s1).all()) and bool((p3 == p1).all())


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16"])
def test_repeated_solves_on_a_ragged_grid(prec):
    """Solves on one plan at a ragged size (n = 200, n_p = 256) repeat bit for bit, also after a
    solve at another eps in between: with 4-byte operands the read-out works in the loop's operand
    buffers, whose padded borders must be zero again when the next solve's loop reads them."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n = 200
    g, G = _rand_case(n, 13)
    gd, Gd = to_dev(g), to_dev(G[None])
    plan = F.Plan(n, 1, prec, max_iters=40)
    outs = []
    for eps in (1e-2, 1e-2, 2e-2, 1e-2):
        ph, rep, st = plan.solve(gd, Gd, eps, 40)
        f, psi = plan.potentials()
        assert st == F.FOT_OK, st
        if eps == 1e-2:
            outs.append((ph.clone(), f.clone(), psi.clone(), rep.err_a_history.copy(), rep.dual.copy()))
    plan.close()
    for k, o in enumerate(outs[1:]):
        assert bool((o[0] == outs[0][0]).all()) and bool((o[1] == outs[0][1]).all()), k
        assert bool((o[2] == outs[0][2]).all()), k
        assert np.array_equal(o[3], outs[0][3]) and np.array_equal(o[4], outs[0][4]), k


def test_potentials_roundtrip():
    import torch
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n = 80
    g, G = _rand_case(n, 6)
    plan = F.Plan(n, 1, "f64", max_iters=20)
    plan.solve(to_dev(g), to_dev(G[None]), 1e-2, 20)
    f, psi = plan.potentials()
    f2 = torch.full_like(f, 0.25)
    plan.set_potentials(f2, psi)
    f3, psi3 = plan.potentials()
    assert bool((f3 == f2).all()) and bool((psi3 == psi).all())
    assert f3.shape == (1, n, n) and f3.dtype == torch.float64


@pytest.mark.parametrize("bad", ["negative", "nan", "zero", "eps", "iters"])
def test_invalid_inputs(bad):
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n = 64
    g, G = _rand_case(n, 1, zeros=False)
    eps, iters = 1e-2, 5
    if bad == "negative":
        G[2, 2] = -1.0
    elif bad == "nan":
        g[1, 1] = np.nan
    elif bad == "zero":
        G[:] = 0.0
    elif bad == "eps":
        eps = -1.0
    elif bad == "iters":
        iters = 6
    plan = F.Plan(n, 1, "f32", max_iters=5)
    with pytest.raises(F.FOTError) as ei:
        plan.solve(to_dev(g), to_dev(G[None]), eps, iters)
    assert ei.value.status == F.FOT_E_INVALID
    # the plan stays usable
    g2, G2 = _rand_case(n, 1, zeros=False)
    plan.solve(to_dev(g2), to_dev(G2[None]), 1e-2, 5)


def test_nonfinite_is_reported():
    """Input and target supports are disjoint half-planes (columns < 32 and >= 32 of 64).
    At eps = 2e-5 the Gibbs factor at distance 32 is exp(-6250), zero even in FP64, so after the
    first V-update a whole column of the target has no contribution and its potential
    overflows: FOT_E_NONFINITE is returned (FP32 and FP64 alike) and the plan stays usable.
    At eps = 5e-4 the factor is exp(-250): below FP32's range, but FP32 operands then store
    Lambda block-normalised with its exponents, and both FP32 and FP64 stay finite."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n = 64
    g = np.zeros((n, n))
    g[:, : n // 2] = 1.0
    G = np.zeros((n, n))
    G[:, n // 2:] = 1.0
    gd, Gd = to_dev(g), to_dev(G[None])
    for prec in ("f32", "f64"):
        plan = F.Plan(n, 1, prec, max_iters=3)
        _, rep, st = plan.solve(gd, Gd, 2e-5, 1, check=False)
        _say(f"case: disjoint supports {prec} eps=2e-5: status {st}, nonfinite {rep.nonfinite}")
        assert st == F.FOT_E_NONFINITE and rep.nonfinite == 1, (prec, st)
        _, rep5, st5 = plan.solve(gd, Gd, 5e-4, 1, check=False)
        _say(f"case: disjoint supports {prec} eps=5e-4: status {st5}, nonfinite {rep5.nonfinite}")
        assert rep5.nonfinite == 0 and st5 != F.FOT_E_NONFINITE, (prec, st5)
        g2, G2 = _rand_case(n, 2, zeros=False)
        plan.solve(to_dev(g2), to_dev(G2[None]), 1e-2, 3)
        plan.close()


def test_tiny_grids():
    for n in (1, 2, 3):
        g = np.arange(1, n * n + 1, dtype=np.float64).reshape(n, n)
        G = np.arange(n * n, 0, -1, dtype=np.float64).reshape(n, n)
        gpu = run_gpu(g, G, 0.1, 5, "f64")
        ref = O.solve_sep(g, G, 0.1, 5)
        e = compare(gpu, ref, g, G, precision="f64")
        assert e["f"] < 1e-10 and e["psi"] < 1e-10 and e["dual"] < 1e-10, (n, e)


def test_annealed_schedule_scaled_lattice():
    """The 2048 lattice workload scaled to n=256: annealed eps 5e-2 -> 2e-3 over 400 its."""
    n, T = 256, 400
    g, G = W.speckle_to_lattice(n)
    e = W.anneal_schedule(5e-2, 2e-3, T)
    _say("case: lattice n=256 annealed f32")
    gpu = run_gpu(g, G, e, T, "f32")
    ref = O.solve_sep(g, G, e, T)
    err = compare(gpu, ref, g, G, precision="f32")
    _say(err)
    assert err["f"] < 1e-6 and err["psi"] < 1e-6 and err["phase"] < 1e-5
    assert err["dual"] < 1e-6


def _workload1_ref(g, G):
    return workload1_ref(g, G)


# potentials and phase, scalars, and the final row-marginal L1 the read-out must reach.  FP16
# carries three more significand bits than BF16 (its narrower exponent range is what the
# range checks watch), so BF16's stated 1e-3 bounds its rounding too.
WL1_TOL = {"f32": (1e-6, 1e-6, None), "bf16x3": (1e-5, 1e-5, 1e-5), "bf16": (1e-3, 1e-3, None),
           "f16": (1e-3, 1e-3, None)}


@pytest.mark.parametrize("prec", ["f32", "bf16x3", "bf16", "f16"])
def test_workload1_full_size(prec):
    """1024 x 1024 two-Gaussian -> ellipses and rings, eps 5e-3, 200 its, in every 32- and
    16-bit operand type (the mixed-precision workload is the same images and schedule).
    BF16x3 must also reach a final marginal error far below BF16's floor (~8e-4)."""
    wl = W.workload(1)
    g, G = wl.images()
    _say(f"case: twogauss_to_shapes n=1024 {prec} 200 it")
    gpu = run_gpu(g, G, 5e-3, 200, prec)
    _say("gpu done; oracle running")
    ref = _workload1_ref(g, G[0])
    e = compare(gpu, ref, g, G[0], precision=prec)
    _say(e)
    tol, stol, err_max = WL1_TOL[prec]
    assert e["f"] < tol and e["psi"] < tol, e
    assert e["hist_a"] <= 1 and e["err_a"] <= 1, e
    assert e["phase"] < tol, e
    assert e["dual"] < stol and e["cost"] < stol, e
    if err_max is not None:
        assert gpu["rep"].err_a[0] < err_max, gpu["rep"].err_a[0]


@pytest.mark.parametrize("profile", [False, True])
def test_graph_replays_match_eager(profile):
    """The HIP-graph replay of the iteration loop equals the eager launches bit for bit, on
    every replay, with unrelated eager GPU work and synchronisations between replays, and
    after a re-capture for a new eps schedule."""
    import torch
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T = 128, 40
    g, G = _rand_case(n, 9)
    gd, Gd = to_dev(g), to_dev(G[None])
    sched = W.anneal_schedule(5e-2, 5e-3, T)
    eager = F.Plan(n, 1, "f32", max_iters=T, graph=False)
    ref = {}
    for key, eps in (("const", 1e-2), ("anneal", sched)):
        ph, rep, _ = eager.solve(gd, Gd, eps, T)
        f, psi = eager.potentials()
        assert rep.graph == 0
        ref[key] = (ph.clone(), f.clone(), psi.clone(), rep.err_a_history.copy(), rep.dual.copy())
    plan = F.Plan(n, 1, "f32", max_iters=T, graph=True, profile=profile)
    for it, key in enumerate(("const", "const", "anneal", "const", "anneal")):
        junk = torch.randn(4096, device=gd.device)
        _ = (junk * junk).sum().item()
        torch.cuda.synchronize()
        ph, rep, _ = plan.solve(gd, Gd, 1e-2 if key == "const" else sched, T)
        f, psi = plan.potentials()
        assert rep.graph == (0 if profile else 1), "unexpected launch path"
        r = ref[key]
        assert bool((ph == r[0]).all()) and bool((f == r[1]).all()) and bool((psi == r[2]).all()), (it, key)
        assert np.array_equal(rep.err_a_history, r[3]) and np.array_equal(rep.dual, r[4]), (it, key)
        if profile:
            # the iteration kernels only: two launches per half-step
            assert rep.n_contract == 4 * T and rep.ms_contract > 0


def test_no_history_flag_changes_nothing_else():
    """FOT_FLAG_NO_HISTORY skips the per-iteration marginal errors: the history is NaN and the
    potentials, phase and final report values are bit-identical to a run with the history."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T = 130, 25
    g, G = _rand_case(n, 21)
    gd, Gd = to_dev(g), to_dev(G[None])
    for prec in ("f32", "bf16"):
        runs = []
        for hist in (True, False):
            plan = F.Plan(n, 1, prec, max_iters=T, history=hist)
            ph, rep, _ = plan.solve(gd, Gd, 1e-2, T)
            f, psi = plan.potentials()
            plan.close()
            runs.append((ph, f, psi, rep))
        (p1, f1, s1, r1), (p2, f2, s2, r2) = runs
        _say(f"case: no-history {prec}: final err_a {r1.err_a[0]:.3e} / {r2.err_a[0]:.3e}")
        assert bool((p1 == p2).all()) and bool((f1 == f2).all()) and bool((s1 == s2).all())
        assert r1.err_a[0] == r2.err_a[0] and r1.err_b[0] == r2.err_b[0] and r1.dual[0] == r2.dual[0]
        assert np.all(np.isfinite(r1.err_a_history)) and np.all(np.isnan(r2.err_a_history))
        assert np.all(np.isnan(r2.err_b_history))


def test_range_loss_is_reported():
    """Below the eps an operand type can represent (1024^2, eps 1e-4, FP32: within one 64-wide
    block the operand exp(psi/eps) spans more than FP32's range, so the entries that dominate the
    Gibbs products underflow), fot_solve still writes its outputs but returns FOT_E_RANGE, with
    err_b (the final plan's column-marginal L1 evaluated in FP64) far above FP32's level; the same
    case in FP64 operands is accurate and returns FOT_OK."""
    from paper_2512_19072_amd import fot as F
    n, T, eps = 1024, 50, 1e-4
    g, G = W.twogauss_to_shapes(n)
    _say("case: twogauss n=1024 eps=1e-4 f32 vs f64, 50 it")
    plan = F.Plan(n, 1, "f32", max_iters=T)
    from tests.parity_util import to_dev
    gd, Gd = to_dev(g), to_dev(G[None] if G.ndim == 2 else G)
    _, rep, st = plan.solve(gd, Gd, eps, T, check=False)
    msg = F.fot_last_error()          # (the next call on this thread clears it)
    plan.close()
    assert st == F.FOT_E_RANGE, st
    assert "use FOT_F64" in msg, msg
    assert rep.err_b[0] > 1e-5
    plan = F.Plan(n, 1, "f64", max_iters=T)
    _, rep64, st64 = plan.solve(gd, Gd, eps, T, check=False)
    plan.close()
    _say(f"err_b f32 {rep.err_b[0]:.3e}, f64 {rep64.err_b[0]:.3e}")
    assert st64 == F.FOT_OK and rep64.err_b[0] < 1e-12
    # the product check is the larger of err_b and the u-direction probe (none in FP64)
    assert not rep.err_products[0] < rep.err_b[0], (rep.err_products[0], rep.err_b[0])
    assert rep64.err_products[0] == rep64.err_b[0]


def test_small_tiles_flag_reaches_half_the_eps():
    """FOT_FLAG_SMALL_TILES runs a 1024^2 solve with 32-wide operand blocks (64 x 64 tiles holding
    two blocks each): at eps = 1e-4, where 64-wide blocks lose FP32's range
    (test_range_loss_is_reported), FP32 operands then match the oracle."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T, eps = 1024, 40, 1e-4
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    _say("case: FOT_FLAG_SMALL_TILES n=1024 f32 eps=1e-4")
    plan = F.Plan(n, 1, "f32", max_iters=T, small_tiles=True)
    _, rep, st = plan.solve(to_dev(g), to_dev(G[None]), eps, T, check=False)
    f, psi = plan.potentials()
    plan.close()
    assert st == F.FOT_OK, (st, F.fot_last_error())
    gpu = dict(f=f.cpu().numpy(), psi=psi.cpu().numpy(), phase=None, rep=rep)
    ref = O.solve_sep(g, G, eps, T)
    from tests.parity_util import gauge_rel
    a = g ** 2 / np.sum(g ** 2)
    b = G ** 2 / np.sum(G ** 2)
    ef, ep = gauge_rel(gpu["f"][0], ref.f, a), gauge_rel(gpu["psi"][0], ref.psi, b)
    _say(f"f {ef:.2e} psi {ep:.2e} err_b {rep.err_b[0]:.2e}")
    assert ef < 1e-6 and ep < 1e-6, (ef, ep)


@pytest.mark.parametrize("prec,eps", [("f32", 1e-2), ("bf16", 1e-2), ("f32", 5e-4)])
def test_block32_tiles_match_small_tiles_bit_for_bit(prec, eps):
    """32-wide exponent blocks on 64 x 64 tiles (FOT_FLAG_SMALL_TILES where the grid takes 64 x 64
    tiles: four 512^2 targets) against 32 x 32 tiles (chosen for one 512^2 target): the blocks, the
    K order of every sum and the element work are the same, so the potentials and the phase of
    each target are bit-identical (at 5e-4 with the block-normalised Lambda as well)."""
    import torch
    n, T = 512, 30
    cus = torch.cuda.get_device_properties(0).multi_processor_count
    if not (128 <= cus < 512):
        pytest.skip(f"{cus} CUs: the two 512^2 cases would not use the two tile configurations")
    g, G = _rand_case(n, 31)
    _say(f"case: 32-wide blocks n={n} {prec} eps={eps}: 32 x 32 tiles (B=1) against 64 x 64 tiles (B=4)")
    one = run_gpu(g, G, eps, T, prec)
    four = run_gpu(g, np.stack([G] * 4), eps, T, prec, small_tiles=True)
    assert one["status"] == four["status"], (one["status"], four["status"])
    for b in range(4):
        for k in ("f", "psi", "phase"):
            same = (one[k][0] == four[k][b]) | (np.isnan(one[k][0]) & np.isnan(four[k][b]))
            assert same.all(), (b, k, int((~same).sum()))


def test_block32_tiles_with_block_normalised_lambda_at_2048():
    """FOT_FLAG_SMALL_TILES at 2048^2 and eps = 1e-4: 64 x 64 tiles with 32-wide blocks and Lambda
    block-normalised (its raw FP32 band is ~300 px), whose doubled exponent table still fits in
    LDS at this n_p; FP32 potentials against the oracle after a few iterations."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import gauge_rel, to_dev
    n, T, eps = 2048, 6, 1e-4
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    _say(f"case: 32-wide blocks on 64 x 64 tiles, block-normalised Lambda, n={n} f32 eps={eps} T={T}")
    plan = F.Plan(n, 1, "f32", max_iters=T, small_tiles=True)
    _, rep, st = plan.solve(to_dev(g), to_dev(G[None]), eps, T, check=False)
    f, psi = plan.potentials()
    plan.close()
    assert st == F.FOT_OK, (st, F.fot_last_error())
    ref = O.solve_sep(g, G, eps, T)
    a = g ** 2 / np.sum(g ** 2)
    b = G ** 2 / np.sum(G ** 2)
    ef, ep = gauge_rel(f.cpu().numpy()[0], ref.f, a), gauge_rel(psi.cpu().numpy()[0], ref.psi, b)
    _say(f"f {ef:.2e} psi {ep:.2e} err_b {rep.err_b[0]:.2e}")
    assert ef < 1e-6 and ep < 1e-6, (ef, ep)


def test_small_eps_beyond_the_lds_table_is_unsupported():
    """At n = 8192 the block-normalised Gibbs factor's exponent table no longer fits in LDS beside
    the 64 x 64-tile stage buffers: a 32-bit solve at an eps that needs it returns
    FOT_E_UNSUPPORTED before launching anything, and names FOT_F64."""
    import torch
    from paper_2512_19072_amd import fot as F
    n = 8192
    _say("case: n=8192 f32 eps=1e-4 (table beyond LDS)")
    plan = F.Plan(n, 1, "f32", max_iters=1)
    g = torch.ones((n, n), dtype=torch.float64, device="cuda")
    G = torch.ones((1, n, n), dtype=torch.float64, device="cuda")
    _, _, st = plan.solve(g, G, 1e-4, 1, check=False)
    msg = F.fot_last_error()
    plan.close()
    assert st == F.FOT_E_UNSUPPORTED, st
    assert "FOT_F64" in msg, msg


def test_largest_grid_f32_against_f64():
    """n = 8192, the largest grid fot_plan accepts: the Toeplitz table of the Gibbs factor no longer
    fits in LDS beside the stage buffers, so the kernels stage it with the K stages.  Two
    iterations at eps = 5e-2 (raw Lambda) with FP32 operands against the same solve with FP64
    operands: potentials and phase within FP32's 1e-6 (range-normalised, gauge-fixed)."""
    import torch
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import gauge_rel, range_rel
    n, T, eps = 8192, 2, 5e-2
    _say(f"case: n={n} f32 against f64, eps={eps}, T={T}")
    x = (torch.arange(n, dtype=torch.float64, device="cuda") - n / 2) / n
    g = torch.exp(-(x[:, None] ** 2 + x[None, :] ** 2) / (2 * 0.15 ** 2))
    G = torch.exp(-((x[:, None] - 0.1) ** 2 / (2 * 0.2 ** 2) + (x[None, :] + 0.05) ** 2 / (2 * 0.1 ** 2)))[None]
    out = {}
    for prec in ("f64", "f32"):
        plan = F.Plan(n, 1, prec, max_iters=T)
        ph, rep, st = plan.solve(g, G, eps, T)
        f, psi = plan.potentials()
        out[prec] = (f.cpu().numpy()[0], psi.cpu().numpy()[0], ph.cpu().numpy()[0], st)
        plan.close()
        del f, psi, ph
        torch.cuda.empty_cache()
    a = (g ** 2 / (g ** 2).sum()).cpu().numpy()
    b = (G[0] ** 2 / (G[0] ** 2).sum()).cpu().numpy()
    assert out["f32"][3] == F.FOT_OK and out["f64"][3] == F.FOT_OK
    ef = gauge_rel(out["f32"][0], out["f64"][0], a)
    ep = gauge_rel(out["f32"][1], out["f64"][1], b)
    eph = range_rel(out["f32"][2], out["f64"][2])
    _say(f"f {ef:.2e} psi {ep:.2e} phase {eph:.2e}")
    assert ef < 1e-6 and ep < 1e-6 and eph < 1e-6, (ef, ep, eph)


def test_u_direction_range_loss_is_reported():
    """On 129^2 at eps = 5e-4 (32-wide blocks: a quarter of the grid) the potential psi comes to
    span more than FP32 holds within one block from about the 27th iteration, so the u-updates'
    products lose values and the iterates drift from the oracle's while the last V-update's
    column marginal stays at 1e-7.  FOT_E_RANGE at 30 iterations (the in-loop check flags it from
    iteration 18, ahead of the drift; the end-of-solve probe, one more u-direction product in the
    operand type against FP64, sees it too); at 15 the solve is exact and not flagged."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, eps = 129, 5e-4
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    gd, Gd = to_dev(g), to_dev(G[None])
    _say("case: u-direction range loss n=129 f32 eps=5e-4, 30 and 20 iterations")
    plan = F.Plan(n, 1, "f32", max_iters=30)
    _, rep, st = plan.solve(gd, Gd, eps, 30, check=False)
    msg = F.fot_last_error()
    assert st == F.FOT_E_RANGE, (st, rep.err_b[0])
    assert "use FOT_F64" in msg, msg
    assert rep.err_b[0] < 1e-5          # the column marginal alone would not have shown it
    plan.close()
    # the same drift in BF16 operands: its product check reads about 1e-2, above BF16's 5e-3
    plan = F.Plan(n, 1, "bf16", max_iters=30)
    _, rep16, st16 = plan.solve(gd, Gd, eps, 30, check=False)
    plan.close()
    _say(f"bf16 err_b {rep16.err_b[0]:.2e} products {rep16.err_products[0]:.2e}")
    assert st16 == F.FOT_E_RANGE and rep16.err_products[0] > 5e-3, (st16, rep16.err_products[0])
    gpu = run_gpu(g, G, eps, 15, "f32")
    ref = O.solve_sep(g, G, eps, 15)
    e = compare(gpu, ref, g, G, precision="f32")
    _say(e)
    assert e["f"] < 1e-6 and e["psi"] < 1e-6, e
    assert gpu["rep"].range_iter[0] == -1


def test_f16_systematic_underflow_is_reported():
    """FP16's exponent range is narrow: on a 65^2 grid at eps = 5e-3 the operand blocks (32 wide:
    half the grid) span more than it holds, the lost small values bias the fixed point (potentials
    off by several 1e-3) while the last update's column marginal stays near 8e-4, and FP16's own
    bound (5e-4) reports FOT_E_RANGE; at eps = 1e-2 the same grid matches the oracle to 1e-3."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T = 65, 30
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    gd, Gd = to_dev(g), to_dev(G[None])
    _say("case: f16 n=65 eps=5e-3 (range loss) and 1e-2")
    plan = F.Plan(n, 1, "f16", max_iters=T)
    _, rep, st = plan.solve(gd, Gd, 5e-3, T, check=False)
    assert st == F.FOT_E_RANGE and rep.err_b[0] > 5e-4, (st, rep.err_b[0])
    plan.close()
    gpu = run_gpu(g, G, 1e-2, T, "f16")
    ref = O.solve_sep(g, G, 1e-2, T)
    e = compare(gpu, ref, g, G, precision="f16")
    _say(e)
    assert e["f"] < 1e-3 and e["psi"] < 1e-3 and e["phase"] < 1e-3, e


@pytest.mark.parametrize("n,prec,eps", [(256, "f64", 2e-4), (320, "f32", 1e-3), (256, "bf16x3", 1e-3),
                                        (512, "f32", 2e-4), (1024, "f32", 2e-4), (1024, "bf16", 2e-4),
                                        (1024, "bf16x3", 2e-4)])
def test_small_eps_band_skipping(n, prec, eps):
    """At small eps Lambda has entries below the operand type's range: FP64 operands skip the K
    stages whose Lambda block is zero (the band of |i - k| where it is not); the 32-bit and 16-bit
    forms store Lambda block-normalised with its own exponents (down to FP64's underflow, with the
    band widened to match).  The result must still be the oracle's, down to the paper's
    eps = 2e-4 (FP32 from 512^2, where an exponent block spans 1/16 of the grid)."""
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    T = 60
    _say(f"case: band skipping n={n} {prec} eps={eps}")
    gpu = run_gpu(g, G, eps, T, prec)
    ref = O.solve_sep(g, G, eps, T)
    e = compare(gpu, ref, g, G, precision=prec)
    _say({k: (f"{v:.2e}" if isinstance(v, float) else v) for k, v in e.items()})
    tol = {"f64": 1e-10, "f32": 1e-6, "bf16": 1e-3, "bf16x3": 1e-5}[prec]
    assert e["f"] < tol and e["psi"] < tol and e["phase"] < tol, e
    assert gpu["status"] == 0, gpu["status"]


def test_bf16_then_f32_schedule_reaches_f32_error():
    """A precision schedule through the C ABI: 29 BF16 iterations on workload 1 (1024^2, eps 5e-3),
    then the potentials into an FP32 plan and one FP32 iteration from them.  Its final row-marginal
    L1 is no higher than FP32's own after 30 iterations (BF16 alone stays above it, near its
    floor), and its potentials match the oracle's 30-iteration ones to BF16's tolerance."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T, eps = 1024, 30, 5e-3
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    gd, Gd = to_dev(g), to_dev(G[None])
    _say("case: bf16 29 + f32 1 iterations, 1024^2 eps 5e-3")
    p16 = F.Plan(n, 1, "bf16", max_iters=T)
    p32 = F.Plan(n, 1, "f32", max_iters=T)
    e16 = p16.solve(gd, Gd, eps, T)[1].err_a[0]
    e32 = p32.solve(gd, Gd, eps, T)[1].err_a[0]
    p16.solve(gd, Gd, eps, T - 1)
    f, psi = p16.potentials()
    p32.set_potentials(f, psi)
    phase, rep, st = p32.solve(gd, Gd, eps, 1, warm_start=True)
    fs, psis = p32.potentials()
    p16.close()
    p32.close()
    _say(f"err_a: bf16 {e16:.3e}, f32 {e32:.3e}, schedule {rep.err_a[0]:.3e}")
    assert st == F.FOT_OK
    assert rep.err_a[0] <= 1.02 * e32 and e16 > 1.2 * e32, (rep.err_a[0], e32, e16)
    # (the warm-started solve's history holds its one iteration only: potentials are compared)
    from tests.parity_util import gauge_rel
    ref = O.solve_sep(g, G, eps, T)
    a = g ** 2 / np.sum(g ** 2)
    b = G ** 2 / np.sum(G ** 2)
    ef = gauge_rel(fs.cpu().numpy()[0], ref.f, a)
    ep = gauge_rel(psis.cpu().numpy()[0], ref.psi, b)
    _say(f"f {ef:.2e} psi {ep:.2e}")
    assert ef < 1e-3 and ep < 1e-3, (ef, ep)


def test_precision_schedule_in_one_solve():
    """The schedule inside the library (fot_plan_desc.tail_precision / tail_iters): 29 BF16 then 1
    FP32 iteration of workload 1 in one fot_solve equals the same schedule chained through two
    plans and fot_potentials bit for bit (each segment builds its operands from psi), in graph
    replays and eager launches alike; with tail_iters >= iters it is an FP32 solve bit for bit."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    n, T, k, eps = 1024, 30, 1, 5e-3
    g, G = W.twogauss_to_shapes(n)
    G = G if G.ndim == 2 else G[0]
    gd, Gd = to_dev(g), to_dev(G[None])
    _say("case: schedule bf16 29 + f32 1 in one solve, 1024^2 eps 5e-3")
    p16 = F.Plan(n, 1, "bf16", max_iters=T)
    p32 = F.Plan(n, 1, "f32", max_iters=T)
    p16.solve(gd, Gd, eps, T - k)
    f, psi = p16.potentials()
    p32.set_potentials(f, psi)
    ph_c, rep_c, _ = p32.solve(gd, Gd, eps, k, warm_start=True)
    f_c, psi_c = p32.potentials()
    ph_32, rep_32, _ = p32.solve(gd, Gd, eps, T)
    f_32, psi_32 = p32.potentials()
    p16.close()
    p32.close()
    for graph in (True, False):
        ps = F.Plan(n, 1, "bf16", max_iters=T, graph=graph, tail_precision="f32", tail_iters=k)
        for rep_i in range(2):           # a second solve replays the cached graph
            ph, rep, st = ps.solve(gd, Gd, eps, T)
            fs, psis = ps.potentials()
            assert st == F.FOT_OK and rep.graph == (1 if graph else 0)
            assert bool((fs == f_c).all()) and bool((psis == psi_c).all()), (graph, rep_i)
            assert bool((ph == ph_c).all()), (graph, rep_i)
            assert rep.err_a[0] == rep_c.err_a[0] and rep.dual[0] == rep_c.dual[0]
        ps.close()
    _say(f"err_a: schedule {rep.err_a[0]:.3e}, f32 alone {rep_32.err_a[0]:.3e}")
    assert rep.err_a[0] <= 1.02 * rep_32.err_a[0]
    # all iterations in the tail type: an FP32 solve
    pt = F.Plan(n, 1, "bf16", max_iters=T, tail_precision="f32", tail_iters=T + 5)
    ph_t, rep_t, _ = pt.solve(gd, Gd, eps, T)
    f_t, psi_t = pt.potentials()
    pt.close()
    assert bool((f_t == f_32).all()) and bool((psi_t == psi_32).all()) and bool((ph_t == ph_32).all())
    assert np.array_equal(rep_t.err_a_history, rep_32.err_a_history)
    # against the oracle's 30 iterations: BF16's tolerance (the last iteration is FP32's)
    from tests.parity_util import gauge_rel
    ref = O.solve_sep(g, G, eps, T)
    a, b = O.normalise(g), O.normalise(G)
    ef = gauge_rel(fs.cpu().numpy()[0], ref.f, a)
    ep = gauge_rel(psis.cpu().numpy()[0], ref.psi, b)
    _say(f"f {ef:.2e} psi {ep:.2e}")
    assert ef < 1e-3 and ep < 1e-3, (ef, ep)


@pytest.mark.parametrize("head,tail,n,k", [("bf16", "f32", 200, 3), ("f16", "bf16x3", 130, 2), ("bf16", "f64", 72, 4)])
def test_precision_schedule_ragged(head, tail, n, k):
    """Schedules on ragged grids (each type's own padding and tiles share the plan) against the
    oracle to the head type's tolerance, with the final iterations' type doing the range check."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev, gauge_rel
    T, eps = 40, 1e-2
    g, G = _rand_case(n, 70 + n)
    _say(f"case: schedule {head} -> {tail} n={n} k={k}")
    ps = F.Plan(n, 1, head, max_iters=T, tail_precision=tail, tail_iters=k)
    ph, rep, st = ps.solve(to_dev(g), to_dev(G[None]), eps, T)
    f, psi = ps.potentials()
    ps.close()
    assert st == F.FOT_OK
    ref = O.solve_sep(g, G, eps, T)
    e = max(gauge_rel(f.cpu().numpy()[0], ref.f, O.normalise(g)),
            gauge_rel(psi.cpu().numpy()[0], ref.psi, O.normalise(G)))
    _say(f"  potentials {e:.2e}")
    assert e < 1e-3


def test_precision_schedule_rejections():
    from paper_2512_19072_amd import fot as F
    for kw, status in ((dict(precision="f32", tail_precision="f32", tail_iters=1), F.FOT_E_INVALID),
                       (dict(precision="f64", tail_precision="f32", tail_iters=1), F.FOT_E_UNSUPPORTED),
                       (dict(precision="bf16", tail_precision="f32", tail_iters=1, checkpoint_every=5),
                        F.FOT_E_UNSUPPORTED),
                       (dict(precision="f64", tail_precision="f32", tail_iters=1, cfot=True), F.FOT_E_UNSUPPORTED),
                       (dict(precision="bf16", tail_precision=9, tail_iters=1), F.FOT_E_INVALID),
                       (dict(precision="bf16", tail_precision="f32", tail_iters=-1), F.FOT_E_INVALID)):
        prec = kw.pop("precision")
        with pytest.raises(F.FOTError) as ei:
            F.Plan(64, 1, prec, max_iters=10, **kw)
        assert ei.value.status == status, (kw, ei.value)


@pytest.mark.parametrize("n,B,prec", [(64, 1, "f32"), (100, 1, "f32"), (128, 2, "f32"), (200, 1, "f32"),
                                      (256, 1, "f32"), (128, 1, "bf16"), (130, 2, "bf16"), (96, 1, "f16")])
def test_small_grids_against_oracle(n, B, prec):
    """Grids whose 64 x 64 tiles would leave most compute units idle run on 32 x 32 tiles with
    32-wide exponent blocks: potentials and phase of target 0 against the oracle, ragged sides
    included (100, 130, 200: a partial last tile and K stage)."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    _say(f"case: small grid n={n} B={B} {prec}")
    g, G = _rand_case(n, 200 + n)
    Gs = np.stack([G * (1.0 + 0.1 * b) + 0.01 * b for b in range(B)])
    plan = F.Plan(n, B, prec, max_iters=30)
    ph, rep, st = plan.solve(to_dev(g), to_dev(Gs), 1e-2, 30, check=False)
    f, psi = plan.potentials()
    out = dict(phase=ph.cpu().numpy(), f=f.cpu().numpy(), psi=psi.cpu().numpy(), rep=rep)
    plan.close()
    assert st == F.FOT_OK, st
    ref = O.solve_sep(g, Gs[0], 1e-2, 30)
    e = compare(out, ref, g, Gs[0], precision=prec)
    tol = {"f32": 1e-6, "bf16": 1e-3, "f16": 1e-3}[prec]
    assert e["f"] < tol and e["psi"] < tol and e["phase"] < tol, e


def test_f64_range_boundary():
    """FP64 operands on the 257^2 two-Gaussian workload at eps = 1e-4: the products keep every term
    that matters through 100 iterations (FOT_OK, within 1e-10 of the oracle, whose exact log-sum-
    exp form engages from about iteration 130), and by 200 iterations some outputs have lost their
    terms to underflow: FOT_E_RANGE, reported at the first iteration whose bound crossed the level,
    with potentials that are indeed off the oracle's."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev, gauge_rel
    n, eps = 257, 1e-4
    g, G = W.twogauss_to_shapes(n)
    gd, Gd = to_dev(g), to_dev(G[None])
    a, b = O.normalise(g), O.normalise(G)
    _say("case: f64 range boundary 257^2 eps 1e-4, 100 and 200 iterations")
    plan = F.Plan(n, 1, "f64", max_iters=200)
    _, rep, st = plan.solve(gd, Gd, eps, 100, check=False)
    f, psi = plan.potentials()
    ref = O.solve_sep(g, G, eps, 100)
    e = max(gauge_rel(f.cpu().numpy()[0], ref.f, a), gauge_rel(psi.cpu().numpy()[0], ref.psi, b))
    _say(f"  T=100: status {st}, range_loss {rep.range_loss[0]:.2e}, potentials {e:.2e}")
    assert st == F.FOT_OK and rep.range_iter[0] == -1 and e < 1e-10
    _, rep, st = plan.solve(gd, Gd, eps, 200, check=False)
    f, psi = plan.potentials()
    plan.close()
    ref = O.solve_sep(g, G, eps, 200)
    e = max(gauge_rel(f.cpu().numpy()[0], ref.f, a), gauge_rel(psi.cpu().numpy()[0], ref.psi, b))
    _say(f"  T=200: status {st}, first iteration {rep.range_iter[0]}, potentials {e:.2e}")
    assert st == F.FOT_E_RANGE and 100 <= rep.range_iter[0] < 200
    assert e > 1e-3


@pytest.mark.parametrize("n,prec,eps,T,reported", [
    (257, "bf16", 2e-4, 30, True), (513, "bf16", 2e-4, 30, True), (1024, "bf16", 1e-4, 30, True),
    (513, "f32", 1e-4, 30, True), (513, "bf16x3", 1e-4, 30, True), (1024, "bf16x3", 1e-4, 30, True),
    (1024, "f32", 2e-4, 60, False), (1024, "bf16x3", 2e-4, 60, False), (1024, "bf16", 2e-4, 60, False)])
def test_mid_trajectory_range_losses_are_reported(n, prec, eps, T, reported):
    """Solves whose iterates lost products mid-trajectory while the final state stayed self-
    consistent (the end-of-solve checks see nothing: potentials off the oracle's by 1e-3 to 3e-2)
    are reported by the in-loop range check; the paper's eps = 2e-4 at 1024^2, where FP32, BF16x3
    and BF16 stay within their tolerances, is not."""
    from paper_2512_19072_amd import fot as F
    from tests.parity_util import to_dev
    g, G = W.twogauss_to_shapes(n)
    _say(f"case: mid-trajectory range n={n} {prec} eps={eps} T={T}")
    plan = F.Plan(n, 1, prec, max_iters=T)
    _, rep, st = plan.solve(to_dev(g), to_dev(G[None]), eps, T, check=False)
    plan.close()
    _say(f"  status {st}, range_loss {rep.range_loss[0]:.2e}, first iteration {rep.range_iter[0]}, "
         f"err_products {rep.err_products[0]:.2e}")
    if reported:
        assert st == F.FOT_E_RANGE and 0 <= rep.range_iter[0] < T
    else:
        assert st == F.FOT_OK and rep.range_iter[0] == -1


@pytest.mark.parametrize("n,B,prec", [(1024, 1, "f32"), (1024, 1, "bf16"), (512, 4, "f32"), (1024, 1, "f64"),
                                       (1000, 1, "f32")])
def test_plan_memory_is_linear_in_pixels(n, B, prec):
    """O(N) memory (Sec. 4, Table 1): a plan's device memory (no tape, no output-beam workspace),
    one allocation, is at most (68 B + 12) bytes per padded pixel for the 32- and 16-bit operand
    types: per target 7 FP64 planes (f, psi, ln b, ln S and the read-out's three scratch planes;
    ln S' is formed again by the read-out, T_x is kept as its one integrated column, the phase goes
    to the caller's array), a fourth read-out plane (T_y) that FP32-sized operands share with the
    loop's two operand planes, and those two planes; shared ln a in FP64 and Lambda in the operand
    type (the read-out reads Lambda and Lambda o H in FP64 from Toeplitz tables of a few KB).  FP64
    plans reuse the loop's buffers for the read-out: (64 B + 16) bytes.  A 1024^2 FP32 plan stays
    within 80 MiB."""
    import torch
    from paper_2512_19072_amd import fot as F
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    plan = F.Plan(n, B, prec, max_iters=200)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    plan.close()
    npad = -(-n // 256) * 256
    per_px = (64 * B + 16) if prec == "f64" else (68 * B + 12)
    bound = per_px * npad * npad + (4 << 20)
    _say(f"plan {n}^2 x {B} {prec}: {used / 2**20:.1f} MiB (bound {bound / 2**20:.1f} MiB)")
    assert used <= bound
    if (n, B, prec) == (1024, 1, "f32"):
        assert used <= 80 << 20
