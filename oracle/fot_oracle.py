"""FP64 CPU oracle for Fast Optimal Transport (FOT) beam shaping (arXiv 2512.19072).

TEST INFRASTRUCTURE ONLY.  This package is the slow, plain reference that the GPU
library is checked against.  Only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import it; the library and its Python binding never do, and this
file imports nothing from them.

What is computed (the paper's notation; p = (j, k) input pixel, q = (L, M) target pixel):

* intensities a = g^2 / sum g^2 and b = G^2 / sum G^2 (marginals of one plan, Sec. 2,
  Eq. 2; the unit-mass normalisation is this package's reading of the paper).
* cost c_pq = ((j-L)^2 + (k-M)^2) / (2 n^2) (Sec. 2, Eq. 3), separable through
  H_jK = (j-K)^2 / (2 n^2) and the Gibbs factor Lambda = exp(-H / eps) (Sec. 3, after Eq. 6).
* Sinkhorn-Knopp scaling (Sec. 3, Eq. 7-8; Algorithm 1) started from u = V = 1/n^2,
  carried in log form: f = eps ln u, psi = eps ln V.  One iteration is a u-update
  followed by a V-update; a fixed number of iterations is run (Sec. 3, text after
  Algorithm 1).  A per-iteration eps schedule is accepted; the potentials are carried
  across eps changes.
* plan Gamma = u K V (Sec. 3, Eq. 6), its marginal L1 errors, the entropic dual value
  D = <f, a> + <psi, b> - eps sum(Gamma) and the transport cost <Gamma, c> (Sec. 2, Eq. 2).
* phase gradients from the duals (Sec. 3, Eq. 9-10), i.e. the first moments of the
  plan divided by the input intensity (Sec. 2, Eq. 4-5), and their integration by the
  trapezoid rule (Sec. 2, text after Eq. 5).
* the reverse-mode derivative of (D, phase) with respect to the target amplitudes G,
  through the unrolled iterations.
* the unregularised OT cost by linear programming (Sec. 2, Eq. 2) for brute-force checks.

Two levels:

O1 ``solve_dense``  the definition written out: the full N x N cost and log-sum-exp over
                    every pixel pair (N = n^2; practical for n <= 32).
O2 ``solve_sep``    the same iteration with every N x N contraction replaced by the exact
                    separable identity K.V = Lambda . V . Lambda (Sec. 3, Eq. 7).  Each of
                    the two per-axis products is, by definition, a log-sum-exp over one index
                    of ln Lambda = -H / eps plus the log-operand; ``sep_log_apply_exact``
                    writes exactly that (chunked, no shifted exponentials, any range).  The
                    fast evaluation ``sep_log_apply`` shifts by the row maximum before the
                    first product and by the column maximum before the second (two FP64
                    matrix products), and checks its own sums: a shifted sum below e^-690
                    could be missing terms lost to FP64 underflow (each off by less than
                    e^-744 after the shift), so each line holding one is re-evaluated by
                    its exact log-sum-exp (with weights, the whole contraction is).  The shifted form is practical at n = 1024.

Readings of the paper used here (where it is silent, garbled or ambiguous):

R1  a and b are normalised to unit mass.
R3  u^0 = V^0 = 1/n^2, one iteration = u-update then V-update, fixed iteration count.
R4  the marginal error is the L1 norm (twice the total variation).  The per-iteration
    history is that of the plan entering each half-step, evaluated with the same eps.
R6  zero-mass pixels have potential -inf; 0 * (-inf) is taken as 0; such pixels carry no
    mass and no gradient.
R7  the phase uses the final u (computed from V_{T-1}) and the final V, literally Eq. 9-10;
    u / a is evaluated as 1 / (Lambda . V_{T-1} . Lambda), which is finite where a = 0.
R8  x <-> j <-> L (row index), y <-> k <-> M (column index), X_L = (L - floor(n/2)) / sqrt(n).
R9  integration: phi_{0,0} = 0, cumulative trapezoid along j at k = 0 with dphi/dx, then
    along k on every row with dphi/dy, step 1/sqrt(n); then the a-weighted mean is removed.
R13 the differentiated scalar is dD * D + <dphi, phi> for caller-supplied weights.
"""
from __future__ import annotations

import math
from dataclasses import dataclass
from typing import Optional

import numpy as np

__all__ = [
    "normalise", "log_intensity", "coords", "cost_1d", "gibbs_1d", "cost_dense", "eps_schedule",
    "solve_dense", "solve_sep", "sep_log_apply", "sep_log_apply_exact", "log_gibbs_1d", "integrate",
    "integrate_adjoint",
    "grad_G", "lp_ot_cost", "entropy", "primal_entropic", "Result",
]

NEG_INF = -np.inf


# ----------------------------------------------------------------------------------
# problem data (Sec. 2)
# ----------------------------------------------------------------------------------

def normalise(amp: np.ndarray) -> np.ndarray:
    """Intensity normalised to unit mass: amp^2 / sum(amp^2) (reading R1 of Eq. 2)."""
    amp = np.asarray(amp, dtype=np.float64)
    inten = amp * amp
    total = inten.sum()
    if not np.isfinite(total) or total <= 0.0:
        raise ValueError("amplitude must be finite with positive total intensity")
    return inten / total


def log_intensity(amp: np.ndarray) -> np.ndarray:
    """ln(amp^2 / sum amp^2) evaluated as 2 ln|amp| - ln sum amp^2.

    A pixel has zero mass exactly when its amplitude is zero (reading R6); a nonzero
    amplitude whose square underflows still has a finite log-intensity."""
    amp = np.asarray(amp, dtype=np.float64)
    total = float(np.sum(amp * amp))
    if not np.isfinite(total) or total <= 0.0:
        raise ValueError("amplitude must be finite with positive total intensity")
    with np.errstate(divide="ignore"):
        return 2.0 * np.log(np.abs(amp)) - math.log(total)


def coords(n: int) -> np.ndarray:
    """Grid coordinate x_j = (j - floor(n/2)) / sqrt(n) (Sec. 2)."""
    return (np.arange(n, dtype=np.float64) - (n // 2)) / math.sqrt(n)


def cost_1d(n: int) -> np.ndarray:
    """H_jK = (j - K)^2 / (2 n^2), the one-axis part of the cost (Sec. 2, after Eq. 5)."""
    i = np.arange(n, dtype=np.float64)
    return (i[:, None] - i[None, :]) ** 2 / (2.0 * n * n)


def gibbs_1d(n: int, eps: float) -> np.ndarray:
    """Lambda_jK = exp(-H_jK / eps) (Sec. 3, after Eq. 6)."""
    return np.exp(-cost_1d(n) / eps)


def log_gibbs_1d(n: int, eps: float) -> np.ndarray:
    """ln Lambda_jK = -H_jK / eps, without forming Lambda (no underflow at any eps)."""
    return -cost_1d(n) / eps


def cost_dense(n: int) -> np.ndarray:
    """Full cost c_pq, p = j*n + k, q = L*n + M (Sec. 2, Eq. 3); N x N, small n only."""
    H = cost_1d(n)
    # c[(j,k),(L,M)] = H[j,L] + H[k,M]
    C = H[:, None, :, None] + H[None, :, None, :]
    return C.reshape(n * n, n * n)


def eps_schedule(eps, iters: int) -> np.ndarray:
    """A length-``iters`` array of eps values (a scalar is repeated)."""
    e = np.atleast_1d(np.asarray(eps, dtype=np.float64))
    if e.size == 1:
        e = np.full(iters, float(e[0]))
    if e.size != iters:
        raise ValueError("eps must be a scalar or have one value per iteration")
    if np.any(~np.isfinite(e)) or np.any(e <= 0):
        raise ValueError("eps must be finite and positive")
    return e


def _log(x: np.ndarray) -> np.ndarray:
    with np.errstate(divide="ignore"):
        return np.log(x)


def _masked_dot(w: np.ndarray, v: np.ndarray) -> float:
    """sum(w * v) with 0 * (-inf) taken as 0 (reading R6)."""
    m = w > 0
    return float(np.sum(w[m] * v[m]))


def entropy(p: np.ndarray) -> float:
    """Shannon entropy -sum p ln p of a probability vector (0 ln 0 = 0)."""
    p = np.asarray(p, dtype=np.float64).ravel()
    m = p > 0
    return float(-np.sum(p[m] * np.log(p[m])))


def primal_entropic(Gamma: np.ndarray, C: np.ndarray, eps: float) -> float:
    """<Gamma, C> + eps sum Gamma (ln Gamma - 1): the primal whose dual is D."""
    m = Gamma > 0
    return float(np.sum(Gamma * C) + eps * np.sum(Gamma[m] * (np.log(Gamma[m]) - 1.0)))


@dataclass
class Result:
    """Outputs of one solve for one target (FP64, [n][n] arrays)."""
    f: np.ndarray            # final input-plane potential eps ln u
    psi: np.ndarray          # final target-plane potential eps ln V
    lnS_last: np.ndarray     # ln(Lambda . V_{T-1} . Lambda), from the final u-update
    err_a_hist: np.ndarray   # [T] row-marginal L1 of the plan entering each u-update
    err_b_hist: np.ndarray   # [T] column-marginal L1 of the plan entering each V-update
    dual_hist: np.ndarray    # [T] dual value after each V-update
    err_a: float             # row-marginal L1 of the final plan
    err_b: float             # column-marginal L1 of the final plan
    dual: float              # <f,a> + <psi,b> - eps sum Gamma of the final plan
    cost: float              # <Gamma, c> of the final plan
    mass: float              # sum Gamma of the final plan
    Tx: np.ndarray           # dphi/dx (Eq. 9)
    Ty: np.ndarray           # dphi/dy (Eq. 10)
    phase: np.ndarray        # integrated phase in cycles (reading R9)
    eps_last: float


# ----------------------------------------------------------------------------------
# integration of the phase gradient (Sec. 2, after Eq. 5; reading R9)
# ----------------------------------------------------------------------------------

def integrate(Tx: np.ndarray, Ty: np.ndarray, a: np.ndarray) -> np.ndarray:
    """Trapezoid integration of (dphi/dx, dphi/dy) with step 1/sqrt(n), a-weighted mean removed."""
    n = Tx.shape[0]
    h = 1.0 / math.sqrt(n)
    col0 = np.zeros(n)
    col0[1:] = np.cumsum(0.5 * h * (Tx[1:, 0] + Tx[:-1, 0]))
    rows = np.zeros((n, n))
    rows[:, 1:] = np.cumsum(0.5 * h * (Ty[:, 1:] + Ty[:, :-1]), axis=1)
    phi = col0[:, None] + rows
    return phi - np.sum(a * phi)


def integrate_adjoint(phibar: np.ndarray, a: np.ndarray):
    """Transpose of :func:`integrate`: maps dL/dphi to (dL/dTx, dL/dTy)."""
    n = phibar.shape[0]
    h = 1.0 / math.sqrt(n)
    pb = phibar - a * phibar.sum()            # transpose of removing the a-weighted mean
    # rows[j, k] = sum_{i<k} h/2 (Ty[j,i] + Ty[j,i+1]);  R[j, i] = sum_{k>i} pb[j, k]
    R = np.cumsum(pb[:, ::-1], axis=1)[:, ::-1] - pb
    Tyb = np.zeros((n, n))
    Tyb[:, :-1] += 0.5 * h * R[:, :-1]
    Tyb[:, 1:] += 0.5 * h * R[:, :-1]
    # col0[j] = sum_{i<j} h/2 (Tx[i,0] + Tx[i+1,0]), added to every k of row j
    cb = pb.sum(axis=1)
    Rc = np.cumsum(cb[::-1])[::-1] - cb
    Txb = np.zeros((n, n))
    Txb[:-1, 0] += 0.5 * h * Rc[:-1]
    Txb[1:, 0] += 0.5 * h * Rc[:-1]
    return Txb, Tyb


# ----------------------------------------------------------------------------------
# O1: the dense definition
# ----------------------------------------------------------------------------------

def _lse(x: np.ndarray, axis: int) -> np.ndarray:
    """log-sum-exp along an axis; an all -inf slice gives -inf."""
    m = np.max(x, axis=axis, keepdims=True)
    m_safe = np.where(np.isfinite(m), m, 0.0)
    with np.errstate(divide="ignore"):
        s = np.log(np.sum(np.exp(x - m_safe), axis=axis, keepdims=True)) + m_safe
    return np.squeeze(s, axis=axis)


def solve_dense(g: np.ndarray, G: np.ndarray, eps, iters: int) -> Result:
    """O1: Sinkhorn on the full N x N cost in log form (Sec. 3, Eq. 6-10; Algorithm 1)."""
    n = g.shape[0]
    e = eps_schedule(eps, iters)
    a = normalise(g).ravel()
    b = normalise(G).ravel()
    la, lb = log_intensity(g).ravel(), log_intensity(G).ravel()
    C = cost_dense(n)
    f = np.full(n * n, e[0] * math.log(1.0 / (n * n)))       # u^0 = 1/n^2
    psi = np.full(n * n, e[0] * math.log(1.0 / (n * n)))     # V^0 = 1/n^2
    err_a_hist = np.zeros(iters)
    err_b_hist = np.zeros(iters)
    dual_hist = np.zeros(iters)
    psi_prev = psi
    for t in range(iters):
        ep = e[t]
        # row marginal of the plan entering this u-update, by its definition
        Gam = np.exp((f[:, None] + psi[None, :] - C) / ep)
        err_a_hist[t] = np.abs(Gam.sum(axis=1) - a).sum()
        # Eq. 7: u = a / (K V)
        f = ep * la - ep * _lse((psi[None, :] - C) / ep, axis=1)
        f[la == NEG_INF] = NEG_INF
        Gam = np.exp((f[:, None] + psi[None, :] - C) / ep)
        err_b_hist[t] = np.abs(Gam.sum(axis=0) - b).sum()
        # Eq. 8: V = b / (K^T u)
        psi_prev = psi
        psi = ep * lb - ep * _lse((f[:, None] - C) / ep, axis=0)
        psi[lb == NEG_INF] = NEG_INF
        Gam = np.exp((f[:, None] + psi[None, :] - C) / ep)
        dual_hist[t] = _masked_dot(a, f) + _masked_dot(b, psi) - ep * Gam.sum()
    ep = e[-1]
    Gam = np.exp((f[:, None] + psi[None, :] - C) / ep)
    lnS_last = _lse((psi_prev[None, :] - C) / ep, axis=1)       # ln (K V_{T-1})
    X = coords(n)
    XL = np.repeat(X, n)          # X_L for q = L*n + M
    YM = np.tile(X, n)            # Y_M
    # Eq. 9-10 with u/a = 1/(K V_{T-1}) (reading R7)
    Wq = np.exp((psi[None, :] - C) / ep - lnS_last[:, None])
    Tx = (Wq @ XL).reshape(n, n)
    Ty = (Wq @ YM).reshape(n, n)
    a2 = a.reshape(n, n)
    return Result(
        f=f.reshape(n, n), psi=psi.reshape(n, n), lnS_last=lnS_last.reshape(n, n),
        err_a_hist=err_a_hist, err_b_hist=err_b_hist, dual_hist=dual_hist,
        err_a=float(np.abs(Gam.sum(axis=1) - a).sum()),
        err_b=float(np.abs(Gam.sum(axis=0) - b).sum()),
        dual=_masked_dot(a, f) + _masked_dot(b, psi) - ep * float(Gam.sum()),
        cost=float(np.sum(Gam * C)), mass=float(Gam.sum()),
        Tx=Tx, Ty=Ty, phase=integrate(Tx, Ty, a2), eps_last=float(ep),
    )


# ----------------------------------------------------------------------------------
# O2: the separable form, Lambda . V . Lambda with per-line shifts
# ----------------------------------------------------------------------------------

def _rowmax(x: np.ndarray) -> np.ndarray:
    m = np.max(x, axis=1)
    return np.where(np.isfinite(m), m, 0.0)


def _colmax(x: np.ndarray) -> np.ndarray:
    m = np.max(x, axis=0)
    return np.where(np.isfinite(m), m, 0.0)


def _signed_exp_scale(W: np.ndarray, shift: np.ndarray) -> np.ndarray:
    """W * exp(shift) evaluated as sign(W) exp(ln|W| + shift), so 0 * exp(large) stays 0."""
    with np.errstate(divide="ignore"):
        return np.sign(W) * np.exp(np.log(np.abs(W)) + shift)


# A factor in a weight entry: None (Lambda) or "H" (Lambda o H, the cost-weighted factor).
def _factor(n: int, eps: float, kind):
    lam = gibbs_1d(n, eps)
    if kind is None:
        return lam
    if kind == "H":
        return lam * cost_1d(n)
    raise ValueError("factor must be None (Lambda) or 'H' (Lambda o H)")


_LSE_CHUNK = 1 << 22     # elements of one [rows][M][k] block of the exact log-sum-exp


def _lse_pass(X: np.ndarray, lnR: np.ndarray, weights=()):
    """One per-axis product in log form, by its definition.

    ``out[L, k] = ln sum_M exp(X[L, M] + lnR[M, k])`` as a log-sum-exp over M for every
    (L, k): the largest term of each sum is taken out before exponentiating, so the terms
    that matter never underflow, whatever the range of X and lnR.  An all -inf sum gives
    -inf.  For each ``(w, h)`` in ``weights`` (either may be None for 1) also returns the
    weighted mean ``sum_M exp(X[L,M] + lnR[M,k] - out[L,k]) w[L,M] h[M,k]`` (0 where the
    sum is empty)."""
    rows, m = X.shape
    k = lnR.shape[1]
    out = np.empty((rows, k))
    avgs = [np.zeros((rows, k)) for _ in weights]
    step = max(1, _LSE_CHUNK // (m * k))
    for r0 in range(0, rows, step):
        r1 = min(rows, r0 + step)
        T = X[r0:r1, :, None] + lnR[None, :, :]            # [rows][M][k]
        mx = T.max(axis=1)                                  # largest term of each sum
        safe = np.where(np.isfinite(mx), mx, 0.0)
        E = np.exp(T - safe[:, None, :])
        tot = E.sum(axis=1)
        with np.errstate(divide="ignore"):
            out[r0:r1] = np.log(tot) + safe
        for i, (w, h) in enumerate(weights):
            Ew = E if w is None else E * w[r0:r1, :, None]
            if h is not None:
                Ew = Ew * h[None, :, :]
            with np.errstate(invalid="ignore", divide="ignore"):
                avgs[i][r0:r1] = np.where(tot > 0, Ew.sum(axis=1) / np.where(tot > 0, tot, 1.0), 0.0)
    return out, avgs


def sep_log_apply_exact(X: np.ndarray, eps: float, weights=()):
    """The separable contraction of exp(X) by its definition, at any range (Sec. 3, Eq. 7).

    ``lnS[j, k] = ln sum_L sum_M Lambda[j, L] exp(X[L, M]) Lambda[M, k]`` is evaluated as two
    exact per-axis log-sum-exps over ln Lambda = -H / eps: first over M (the second index of
    X), then over L.  For each ``(left, right, w)`` in ``weights`` (``left``/``right``: None
    for Lambda or "H" for Lambda o H; ``w`` an [n][n] weight on X or None) the ratio
    ``(left . (exp(X) * w) . right) / (Lambda . exp(X) . Lambda)`` is returned, formed as a
    weighted mean of each pass's terms (so signed weights cancel at the size of the sum)."""
    n = X.shape[0]
    H = cost_1d(n)
    lnL = log_gibbs_1d(n, eps)
    for left, right, _ in weights:
        if left not in (None, "H") or right not in (None, "H"):
            raise ValueError("factor must be None (Lambda) or 'H' (Lambda o H)")
    # first product: W[L, k] = sum_M exp(X[L, M]) right[M, k]
    lnW, mean1 = _lse_pass(X, lnL, [(w, H if right == "H" else None) for _, right, w in weights])
    # second product: S[j, k] = sum_L left[j, L] W[L, k], written as (W^T . left^T)[k, j]
    # (Lambda and H are symmetric)
    lnST, mean2 = _lse_pass(lnW.T, lnL, [(r.T, H if left == "H" else None)
                                         for r, (left, _, _) in zip(mean1, weights)])
    return lnST.T, [r.T for r in mean2]


# ln of the smallest shifted sum that the row- and column-shifted products accept.  After the
# shifts every factor is at most 1, and a term that FP64 cannot hold exactly (a factor or the
# product below the smallest normal number, e^-708) is off by less than 2^-1074 (about e^-744)
# in absolute value, or is lost only if it was below that; n such terms change a sum of at least
# e^-690 by less than 2 n e^-54 relative, far below FP64 rounding for any grid here.  A line
# with a smaller sum is evaluated by the exact log-sum-exp.
SHIFT_SAFE_LOG = -690.0


def _unsafe_lines(sums: np.ndarray, mass: np.ndarray, axis: int) -> np.ndarray:
    """Lines (along ``axis``) with mass holding a shifted sum below e^SHIFT_SAFE_LOG."""
    with np.errstate(divide="ignore"):
        low = np.log(sums) < SHIFT_SAFE_LOG
    return mass & np.any(low, axis=axis)


def sep_log_apply(X: np.ndarray, eps: float, weights=()):
    """Separable contraction of exp(X) in FP64, with per-line shifts (checked against range).

    Returns ``(lnS, ratios)`` with ``lnS = ln(Lambda . exp(X) . Lambda)`` and, for every entry
    ``(left, right, w)`` of ``weights``, ``ratios[i] = (left . (exp(X) * w) . right) /
    (Lambda . exp(X) . Lambda)`` (``left``/``right``: None for Lambda or "H" for Lambda o H;
    ``w`` may be None for 1).  The first product contracts the second index of X after
    shifting each row by its maximum; the second contracts the first index after shifting
    each column by its maximum.  Row and column shifts come from the positive product, so
    signed weights stay well scaled.  A line with mass whose shifted sums fall below
    e^SHIFT_SAFE_LOG somewhere could be missing terms lost to underflow: such a row of the
    first product (column of the second) is evaluated by its exact log-sum-exp instead, and
    with weights the whole contraction goes to ``sep_log_apply_exact``.
    """
    n = X.shape[0]
    lam = gibbs_1d(n, eps)
    lnL = log_gibbs_1d(n, eps)
    m = _rowmax(X)                                            # per-row shift
    A = np.exp(X - m[:, None])                                # in [0, 1]
    W = A @ lam
    row_mass = np.any(X > -np.inf, axis=1)
    bad_rows = _unsafe_lines(W, row_mass, axis=1)
    if weights and np.any(bad_rows):
        return sep_log_apply_exact(X, eps, weights)
    with np.errstate(divide="ignore"):
        Z = m[:, None] + np.log(W)                            # ln(exp(X) . Lambda)
    if np.any(bad_rows):
        Z[bad_rows] = _lse_pass(X[bad_rows], lnL)[0]
    m2 = _colmax(Z)                                           # per-column shift
    B = np.exp(Z - m2[None, :])
    S = lam @ B
    with np.errstate(divide="ignore"):
        lnS = m2[None, :] + np.log(S)
    bad_cols = _unsafe_lines(S, np.full(n, np.any(row_mass)), axis=0)
    if np.any(bad_cols):
        if weights:
            return sep_log_apply_exact(X, eps, weights)
        # S[j, k] = sum_L Lambda[j, L] exp(Z[L, k]), as (Z^T . Lambda)[k, j] in log form
        lnS[:, bad_cols] = _lse_pass(Z[:, bad_cols].T, lnL)[0].T
    ratios = []
    for left, right, w in weights:
        Aw = A if w is None else A * w
        Ww = Aw @ _factor(n, eps, right)
        Bw = _signed_exp_scale(Ww, m[:, None] - m2[None, :])
        with np.errstate(invalid="ignore", divide="ignore"):
            ratios.append(np.where(S > 0, (_factor(n, eps, left) @ Bw) / S, 0.0))
    return lnS, ratios


def _mass_minus_marginal(m, lnm, d):
    """sum |m exp(d) - m| over pixels of positive marginal m (ln m given): the entering plan's
    pixel mass m e^d is at most the plan's total mass, but e^d alone overflows for tiny m, so
    large d use exp(ln m + d) - m (the same quantity)."""
    small = d < 10.0
    return float(np.sum(m[small] * np.abs(np.expm1(d[small])))
                 + np.sum(np.abs(np.exp(lnm[~small] + d[~small]) - m[~small])))


def _solve_sep_one(a, b, la, lb, e, iters, keep_tape=False, start=None):
    n = a.shape[0]
    if start is None:
        f = np.full((n, n), e[0] * math.log(1.0 / (n * n)))
        psi = np.full((n, n), e[0] * math.log(1.0 / (n * n)))
    else:                                       # continue from given potentials (f, psi)
        f, psi = (np.array(x, dtype=np.float64) for x in start)
    err_a_hist = np.zeros(iters)
    err_b_hist = np.zeros(iters)
    dual_hist = np.zeros(iters)
    tape = [] if keep_tape else None
    am, bm = la > NEG_INF, lb > NEG_INF
    psi_prev = psi
    lnS = None
    lnSp = None
    for t in range(iters):
        ep = e[t]
        # Eq. 7 in log form: f = eps (ln a - ln(Lambda . V . Lambda))
        lnS, _ = sep_log_apply(psi / ep, ep)
        f_new = np.where(am, ep * (la - lnS), NEG_INF)
        # marginal identity: row sums of the entering plan are u_old S = a exp((f_old - f_new)/eps)
        # where a > 0, and exp(f_old/eps + ln S) where a = 0 (nonzero only while f_old is finite)
        with np.errstate(invalid="ignore", over="ignore"):
            err_a_hist[t] = (_mass_minus_marginal(a[am], la[am], (f[am] - f_new[am]) / ep)
                             + np.sum(np.exp(f[~am] / ep + lnS[~am])))
        f = f_new
        # Eq. 8 in log form
        lnSp, _ = sep_log_apply(f / ep, ep)
        psi_new = np.where(bm, ep * (lb - lnSp), NEG_INF)
        with np.errstate(invalid="ignore", over="ignore"):
            err_b_hist[t] = (_mass_minus_marginal(b[bm], lb[bm], (psi[bm] - psi_new[bm]) / ep)
                             + np.sum(np.exp(psi[~bm] / ep + lnSp[~bm])))
        psi_prev, psi = psi, psi_new
        # after a V-update sum(Gamma) = sum(b) = 1
        dual_hist[t] = _masked_dot(a, f) + _masked_dot(b, psi) - ep * float(b.sum())
        if keep_tape:
            tape.append((f, psi, lnS, lnSp, ep))
    return f, psi, psi_prev, lnS, lnSp, err_a_hist, err_b_hist, dual_hist, tape


def _readout(a, b, la, lb, f, psi, lnS_last, lnSp_last, ep):
    """Final plan statistics and Eq. 9-10 for potentials (f, psi) = (f_T, psi_T)."""
    n = a.shape[0]
    X = coords(n)
    am = la > NEG_INF
    ones = np.ones((n, n))
    # ln(Lambda.V_T.Lambda) and the ratios needed for Eq. 9-10 and for <Gamma, c>
    lnS_T, (rx, ry, rcx, rcy) = sep_log_apply(
        psi / ep, ep,
        weights=[(None, None, X[:, None] * ones),      # Lambda diag(X) V Lambda
                 (None, None, X[None, :] * ones),      # Lambda V diag(Y) Lambda
                 ("H", None, None),                    # (Lambda o H) V Lambda
                 (None, "H", None)])                   # Lambda V (Lambda o H)
    # u / a = 1 / S(V_{T-1});  Eq. 9: Tx = u (Lambda diag(X) V Lambda) / a
    scale = np.exp(lnS_T - lnS_last)                   # S(V_T) / S(V_{T-1})
    Tx = rx * scale
    Ty = ry * scale
    row_mass = np.where(am, a * scale, 0.0)            # u_T * S(V_T)
    err_a = float(np.sum(np.abs(row_mass - a)))
    col_mass = np.exp(psi / ep + lnSp_last)        # 0 where psi = -inf
    err_b = float(np.sum(np.abs(col_mass - b)))
    mass = float(row_mass.sum())
    cost = float(np.sum(row_mass * (rcx + rcy)))
    dual = _masked_dot(a, f) + _masked_dot(b, psi) - ep * mass
    return Tx, Ty, err_a, err_b, mass, cost, dual


def solve_sep(g: np.ndarray, G: np.ndarray, eps, iters: int, start=None):
    """O2: separable FOT (Algorithm 1) in FP64.  ``G`` may be [n][n] or [B][n][n].

    ``start = (f, psi)`` continues from given potentials instead of u = V = 1/n^2 (single
    target only).  Returns a :class:`Result` for a single target, or a list of them for a batch.
    """
    G = np.asarray(G, dtype=np.float64)
    if G.ndim == 3:
        assert start is None, "start potentials are per target"
        return [solve_sep(g, Gb, eps, iters) for Gb in G]
    e = eps_schedule(eps, iters)
    a = normalise(g)
    b = normalise(G)
    la, lb = log_intensity(g), log_intensity(G)
    f, psi, psi_prev, lnS, lnSp, ea, eb, dh, _ = _solve_sep_one(a, b, la, lb, e, iters, start=start)
    Tx, Ty, err_a, err_b, mass, cost, dual = _readout(a, b, la, lb, f, psi, lnS, lnSp, e[-1])
    return Result(f=f, psi=psi, lnS_last=lnS, err_a_hist=ea, err_b_hist=eb, dual_hist=dh,
                  err_a=err_a, err_b=err_b, dual=dual, cost=cost, mass=mass,
                  Tx=Tx, Ty=Ty, phase=integrate(Tx, Ty, a), eps_last=float(e[-1]))


# ----------------------------------------------------------------------------------
# reverse mode through the unrolled iterations (O2 form)
# ----------------------------------------------------------------------------------

def _Kt_weighted(h_over_eps, w, eps):
    """Return (ln K^T e^{h/eps}, ratio) with ratio = K^T(e^{h/eps} w) / K^T e^{h/eps}.

    K is symmetric and separable, so K^T = K = Lambda (.) Lambda."""
    lnK, (r,) = sep_log_apply(h_over_eps, eps, weights=[(None, None, w)])
    return lnK, r


def grad_G(g: np.ndarray, G: np.ndarray, eps, iters: int, dD: float,
           dphi: Optional[np.ndarray]) -> np.ndarray:
    """d(dD * D + <dphi, phase>)/dG for one target [n][n], by a reverse sweep in FP64.

    Forward: f_t = eps_t (ln a - ln S(psi_{t-1})), psi_t = eps_t (ln b - ln S'(f_t)); the phase
    uses Tx = S_x(psi_T) / S(psi_{T-1}) (Eq. 9) and Ty likewise (Eq. 10); D = <f_T,a> + <psi_T,b>
    - eps_T sum Gamma, with sum Gamma = sum b after a V-update.  b = G^2 / sum G^2.
    """
    n = g.shape[0]
    e = eps_schedule(eps, iters)
    a = normalise(g)
    Gd = np.asarray(G, dtype=np.float64)
    Z = float(np.sum(Gd * Gd))
    b = Gd * Gd / Z
    la, lb = log_intensity(g), log_intensity(Gd)
    am, bm = la > NEG_INF, lb > NEG_INF
    f, psi, psi_prev, lnS, lnSp, _, _, _, tape = _solve_sep_one(a, b, la, lb, e, iters, keep_tape=True)
    X = coords(n)
    ones = np.ones((n, n))

    psibar = np.where(bm, dD * b, 0.0)                 # from <psi_T, b>
    fbar = np.where(am, dD * a, 0.0)                   # from <f_T, a>
    bbar_explicit = np.where(bm, dD * psi, 0.0)        # from <psi_T, b> (b explicit)
    lbbar = np.zeros((n, n))

    # phase: Tx = Sx(psi_T)/S(psi_{T-1}), Ty likewise
    psibar_prev = np.zeros((n, n))
    if dphi is not None:
        epT = e[-1]
        lnS_T, (rx, ry) = sep_log_apply(psi / epT, epT,
                                        weights=[(None, None, X[:, None] * ones),
                                                 (None, None, X[None, :] * ones)])
        scale = np.exp(lnS_T - lnS)
        Tx, Ty = rx * scale, ry * scale
        Txb, Tyb = integrate_adjoint(np.asarray(dphi, dtype=np.float64), a)
        # psibar_T += (V_T / eps) [X K^T(Txb / S_{T-1}) + Y K^T(Tyb / S_{T-1})]
        h = -lnS                                          # 1/S_{T-1} = e^{h}
        lnKx, rxb = _Kt_weighted(h, Txb, epT)
        lnKy, ryb = _Kt_weighted(h, Tyb, epT)
        VT = psi / epT
        psibar = psibar + np.where(
            bm, (X[:, None] * np.exp(VT + lnKx) * rxb + X[None, :] * np.exp(VT + lnKy) * ryb) / epT,
            0.0)
        # psibar_{T-1} += -(V_{T-1}/eps) K^T((Txb Tx + Tyb Ty) / S_{T-1})
        lnKp, rp = _Kt_weighted(h, Txb * Tx + Tyb * Ty, epT)
        psibar_prev = np.where(bm, -np.exp(psi_prev / epT + lnKp) * rp / epT, 0.0)

    for t in range(iters - 1, -1, -1):
        f_t, psi_t, lnS_t, lnSp_t, ep = tape[t]
        # V-update reverse: psi_t = eps (lb - lnS'(f_t))
        lbbar += np.where(bm, ep * psibar, 0.0)
        lnK, r = _Kt_weighted(-lnSp_t, psibar, ep)
        fbar = fbar + np.where(am, -np.exp(f_t / ep + lnK) * r, 0.0)
        # u-update reverse: f_t = eps (la - lnS(psi_{t-1}))
        psi_tm1 = tape[t - 1][1] if t > 0 else None
        if t > 0:
            lnK2, r2 = _Kt_weighted(-lnS_t, fbar, ep)
            psibar = np.where(bm, -np.exp(psi_tm1 / ep + lnK2) * r2, 0.0)
            if t == iters - 1:
                psibar = psibar + psibar_prev
        fbar = np.zeros((n, n))
    # b = G^2 / Z:  Gbar = (2G/Z)(bbar - <bbar, b>),  bbar = lbbar / b + bbar_explicit
    inner = float(lbbar.sum() + np.sum(bbar_explicit * b))
    with np.errstate(divide="ignore", invalid="ignore"):
        Gbar = np.where(Gd != 0, 2.0 * lbbar / np.where(Gd != 0, Gd, 1.0), 0.0)
    Gbar = Gbar + (2.0 * Gd / Z) * (bbar_explicit - inner)
    return Gbar


# ----------------------------------------------------------------------------------
# brute force: the unregularised problem as a linear programme (Sec. 2, Eq. 2)
# ----------------------------------------------------------------------------------

def lp_ot_cost(a: np.ndarray, b: np.ndarray, C: np.ndarray) -> float:
    """min <Gamma, C> s.t. Gamma >= 0, row sums a, column sums b (HiGHS)."""
    from scipy.optimize import linprog
    a = np.asarray(a, dtype=np.float64).ravel()
    b = np.asarray(b, dtype=np.float64).ravel()
    N, M = a.size, b.size
    rows = np.zeros((N, N * M))
    for p in range(N):
        rows[p, p * M:(p + 1) * M] = 1.0
    cols = np.zeros((M, N * M))
    for q in range(M):
        cols[q, q::M] = 1.0
    A_eq = np.vstack([rows, cols])
    b_eq = np.concatenate([a, b])
    res = linprog(C.ravel(), A_eq=A_eq, b_eq=b_eq, bounds=(0, None), method="highs")
    if res.status != 0:
        raise RuntimeError("LP failed: " + res.message)
    return float(res.fun)
