"""Planted mistakes in the oracle (on the CPU) must each fail at least one pin.

Each case replaces one oracle routine with a plausibly wrong variant for the duration of
the test and checks that a pin from test_oracle_pins raises.  This shows the pins are
strong enough to catch a dropped factor, a sign error, a transposed operand, a wrong
integration step or a missing normalisation.
"""
import numpy as np
import pytest

import oracle.fot_oracle as F
from tests import test_oracle_pins as P


def _wrong_cost(n):
    i = np.arange(n, dtype=np.float64)
    return (i[:, None] - i[None, :]) ** 2 / (n * n)            # dropped the 1/2


def _wrong_coords(n):
    return -(np.arange(n, dtype=np.float64) - (n // 2)) / np.sqrt(n)   # sign flip


def _wrong_normalise(amp):
    amp = np.asarray(amp, dtype=np.float64)
    return amp / amp.sum()                                      # amplitude, not intensity


def _wrong_log_intensity(amp):
    amp = np.asarray(amp, dtype=np.float64)
    with np.errstate(divide="ignore"):
        return np.log(np.abs(amp)) - np.log(np.abs(amp).sum())  # amplitude, not intensity


_real_sep = F.sep_log_apply


def _transposed_sep(X, eps, weights=()):
    return _real_sep(X.T, eps, weights)                          # transposed operand


_real_integrate = F.integrate


def _wrong_step_integrate(Tx, Ty, a):
    return _real_integrate(Tx, Ty, a) * 2.0                      # wrong step length


def _no_mean_adjoint(phibar, a):
    return _real_adjoint(phibar, np.zeros_like(a))               # forgot the mean removal


_real_adjoint = F.integrate_adjoint


CASES = [
    ("cost_1d", _wrong_cost, [P.test_product_measures_factorise]),
    ("coords", _wrong_coords, [P.test_gaussian_to_gaussian_affine_map,
                                P.test_phase_matches_continuum_closed_form]),
    ("log_intensity", _wrong_log_intensity, [P.test_two_by_two_first_iteration]),
    ("normalise", _wrong_normalise, [P.test_two_by_two_first_iteration]),
    ("sep_log_apply", _transposed_sep, [lambda: P.test_dense_equals_separable(7, 1e-2)]),
    # the range guard of the shifted products removed (never fall back to the exact form)
    ("SHIFT_SAFE_LOG", -np.inf, [P.test_guarded_oracle_stays_finite_past_the_shifted_range]),
    ("integrate", _wrong_step_integrate, [P.test_phase_matches_continuum_closed_form]),
    ("integrate_adjoint", _no_mean_adjoint, [P.test_integrate_adjoint_is_transpose]),
]


@pytest.mark.parametrize("name,bad,pins", CASES, ids=[c[0] for c in CASES])
def test_planted_mistake_is_caught(monkeypatch, name, bad, pins):
    monkeypatch.setattr(F, name, bad)
    monkeypatch.setattr(P.O, name, bad, raising=False)
    for pin in pins:
        with pytest.raises((AssertionError, ValueError)):
            pin()
