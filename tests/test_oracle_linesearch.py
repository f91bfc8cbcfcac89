"""Pins of the oracle's Moré–Thuente line search (no GPU).

* the strong Wolfe conditions hold at every 'converged' exit;
* on a quadratic the first interpolation lands on the exact minimiser, from
  either side (an overshoot that brackets the minimum, and an extrapolation
  from a point short of it, both computed by hand);
* exits without a Wolfe point report the status and keep every trial.

Not a pin: the comparison with scipy's port of MINPACK-2 DCSRCH
(``scalar_search_wolfe1``).  The oracle follows the same reference form of
the method, so agreement only guards against regressions in this module.
"""
import math

import numpy as np
import pytest
from scipy.optimize._linesearch import scalar_search_wolfe1

from oracle.linesearch import more_thuente

FTOL, GTOL = 1e-4, 1e-2


def _wrap(fun, dfun, log=None):
    def phi(s):
        if log is not None:
            log.append(s)
        return fun(s), dfun(s), None
    return phi


FUNCS = {
    "quadratic": (lambda s: (s - 3.7) ** 2 - 1.0, lambda s: 2 * (s - 3.7)),
    "quartic": (lambda s: (s - 0.3) ** 4 + 0.1 * (s - 0.3) ** 2 - 0.5 * s,
                lambda s: 4 * (s - 0.3) ** 3 + 0.2 * (s - 0.3) - 0.5),
    "mt1": (lambda s: -s / (s * s + 2.0), lambda s: (s * s - 2.0) / (s * s + 2.0) ** 2),
    "mt2": (lambda s: (s + 0.004) ** 5 - 2 * (s + 0.004) ** 4,
            lambda s: 5 * (s + 0.004) ** 4 - 8 * (s + 0.004) ** 3),
    "sine": (lambda s: -math.sin(s) - 0.1 * s, lambda s: -math.cos(s) - 0.1),
    "steep": (lambda s: math.exp(-5 * s) + s * s, lambda s: -5 * math.exp(-5 * s) + 2 * s),
}


@pytest.mark.parametrize("name", list(FUNCS))
@pytest.mark.parametrize("stp0", [1e-3, 1e-1, 1.0, 10.0])
def test_p9_strong_wolfe_on_exit(name, stp0):
    f, df = FUNCS[name]
    f0, g0 = f(0.0), df(0.0)
    assert g0 < 0
    res = more_thuente(_wrap(f, df), f0, g0, stp=stp0, ftol=FTOL, gtol=GTOL, maxfev=40)
    assert res.status == "converged", res
    assert res.f <= f0 + FTOL * res.stp * g0
    assert abs(res.g) <= GTOL * abs(g0)


def test_p9_quadratic_exact_minimiser_after_one_interpolation():
    a, b, c = 2.5, 0.37, -4.0
    f = lambda s: a * (s - b) ** 2 + c
    df = lambda s: 2 * a * (s - b)
    log = []
    res = more_thuente(_wrap(f, df, log), f(0.0), df(0.0), stp=1.0, ftol=FTOL, gtol=GTOL)
    assert res.status == "converged"
    assert res.nfev == 2          # trial 1.0 overshoots, cubic = exact quadratic minimiser
    assert abs(res.stp - b) <= 1e-12


def test_p9_first_step_accepted_when_wolfe():
    f = lambda s: (s - 1.0) ** 2
    df = lambda s: 2 * (s - 1.0)
    res = more_thuente(_wrap(f, df), f(0.0), df(0.0), stp=1.0)
    assert res.nfev == 1 and res.stp == 1.0


def test_maxfev_exit_reports_status():
    f, df = FUNCS["mt2"]
    res = more_thuente(_wrap(f, df), f(0.0), df(0.0), stp=1e-3, maxfev=2)
    assert res.status in ("maxfev", "converged")
    assert res.nfev <= 2


def test_rejects_ascent_direction():
    with pytest.raises(ValueError):
        more_thuente(_wrap(lambda s: s, lambda s: 1.0), 0.0, 1.0)


def test_p9_extrapolation_step_by_hand():
    """phi(s) = (s - 3)^2 - 9 from s = 1: phi = -5, phi' = -4 (sufficient
    decrease, no curvature: gtol is tiny).  Lower value with a smaller slope
    of the same sign and no bracket: the cubic through (0, 0, -6) and
    (1, -5, -4) has theta = 3 (0 + 5) / 1 - 6 - 4 = 5, gamma = -1 (the
    square root of 25/36 - 24/36 times 6, negated since the step increased),
    p = 8, q = -4, r = -2, so the cubic step is 1 + (-2)(0 - 1) = 3; the
    secant step on the derivatives is 1 + (-4 / 2)(-1) = 3 as well.  The
    second trial is therefore the exact minimiser 3, where phi' = 0."""
    f = lambda s: (s - 3.0) ** 2 - 9.0
    df = lambda s: 2.0 * (s - 3.0)
    log = []
    res = more_thuente(_wrap(f, df, log), 0.0, -6.0, stp=1.0, ftol=FTOL, gtol=1e-12, maxfev=5)
    assert log == [1.0, 3.0]
    assert res.status == "converged" and res.stp == 3.0 and res.f == -9.0


def test_p9_maxfev_exit_by_hand():
    """The same function with one evaluation allowed: the trial s = 1 meets
    sufficient decrease but not curvature, so the search stops with status
    'maxfev' at that trial, and the trial list holds exactly it."""
    f = lambda s: (s - 3.0) ** 2 - 9.0
    df = lambda s: 2.0 * (s - 3.0)
    res = more_thuente(_wrap(f, df), 0.0, -6.0, stp=1.0, ftol=FTOL, gtol=1e-12, maxfev=1)
    assert res.status == "maxfev" and res.nfev == 1
    assert [(t[0], t[1], t[2]) for t in res.trials] == [(1.0, -5.0, -4.0)]


@pytest.mark.parametrize("name", list(FUNCS))
@pytest.mark.parametrize("stp0", [1e-3, 1e-1, 1.0, 10.0])
def test_regression_crosscheck_scipy_dcsrch(name, stp0):
    """Regression cross-check, not a pin: scipy's port of the same reference
    form (MINPACK-2 DCSRCH) gives the same trial sequence to rounding."""
    f, df = FUNCS[name]
    ours_log, ref_log = [], []
    amin, amax, xtol = 1e-10, 1e4, 1e-14
    res = more_thuente(_wrap(f, df, ours_log), f(0.0), df(0.0), stp=stp0, ftol=FTOL,
                       gtol=GTOL, xtol=xtol, stpmin=amin, stpmax=amax, maxfev=100)

    def phi(s):
        ref_log.append(("f", s))
        return f(s)

    def dphi(s):
        return df(s)

    # scipy starts from 1.0 unless given old_phi0; reproduce stp0 through it:
    # alpha1 = min(1, 1.01 * 2 * (phi0 - old_phi0) / derphi0)
    old = f(0.0) - stp0 * df(0.0) / (1.01 * 2.0)
    stp, _, _ = scalar_search_wolfe1(phi, dphi, phi0=f(0.0), old_phi0=old if stp0 < 1 else None,
                                     derphi0=df(0.0), c1=FTOL, c2=GTOL, amax=amax, amin=amin,
                                     xtol=xtol)
    if stp0 > 1.0:
        pytest.skip("scipy caps the first step at 1")
    ref_trials = [s for (_, s) in ref_log]
    assert len(ref_trials) == len(ours_log)
    np.testing.assert_allclose(ours_log, ref_trials, rtol=1e-10, atol=1e-14)
    assert stp is not None and abs(stp - res.stp) <= 1e-10 * max(1.0, abs(stp))
