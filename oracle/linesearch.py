"""Moré–Thuente line search, FP64 oracle (test infrastructure only).

Section 2.4 fixes the line search of Step III as the Moré–Thuente method with
function-value tolerance 1e-4, gradient tolerance 1e-2, first trial step 1 and
at most 20 evaluations.  The method (J. J. More and D. J. Thuente, "Line
search algorithms with guaranteed sufficient decrease", ACM TOMS 20(3), 1994)
searches for a step satisfying the strong Wolfe conditions

    phi(stp) <= phi(0) + ftol * stp * phi'(0)      (sufficient decrease)
    |phi'(stp)| <= gtol * |phi'(0)|                (curvature)

keeping an interval of uncertainty [stx, sty], working on the auxiliary
function psi(stp) = phi(stp) - phi(0) - ftol * stp * phi'(0) until a point
with psi <= 0 and phi' >= 0 has been seen, and choosing each new trial by a
safeguarded cubic / quadratic / secant interpolation in four cases.

The authors published the method together with its reference form, the
MINPACK-2 routines DCSRCH (the search: stage switch, convergence and warning
tests, bracket shrinkage by 0.66 with bisection, extrapolation bounds 1.1 and
4.0 of the last step) and DCSTEP (one safeguarded trial step).  This module
follows that reference form operation by operation, because the search's
trial sequence -- and with it every N-GMRES trajectory -- depends on the
exact order of these operations; the GPU library's host-side search follows
the same form for the same reason.  The code is written here from that
description, not copied.

The paper leaves xtol, stpmin and stpmax open; the defaults below
(1e-15, 1e-15, 1e15) are this implementation's stated choice.

Pins (tests/test_oracle_linesearch.py): the strong-Wolfe conditions hold at
every converged exit on analytic functions; on a quadratic the first
interpolation lands on the exact minimiser; with one evaluation allowed, the
exit status and trial are fixed by hand.  A comparison with scipy's DCSRCH
port is kept as a regression cross-check only: it follows the same reference
form, so agreement does not independently pin the method.
"""
from __future__ import annotations

import math

__all__ = ["more_thuente", "LineSearchResult"]

_XTRAPL = 1.1   # lower extrapolation factor (paper's delta_min-style bound)
_XTRAPU = 4.0   # upper extrapolation factor
_P66 = 0.66     # required interval shrink factor before bisection is forced


class LineSearchResult:
    __slots__ = ("stp", "f", "g", "payload", "nfev", "status", "trials")

    def __init__(self, stp, f, g, payload, nfev, status, trials):
        self.stp, self.f, self.g, self.payload = stp, f, g, payload
        self.nfev, self.status, self.trials = nfev, status, trials

    def __repr__(self):
        return (f"LineSearchResult(stp={self.stp!r}, f={self.f!r}, g={self.g!r}, "
                f"nfev={self.nfev}, status={self.status!r})")


def _cubic_minimiser(a, fa, da, b, fb, db):
    """Minimiser of the cubic through (a, fa, da) and (b, fb, db), anchored at a."""
    theta = 3.0 * (fa - fb) / (b - a) + da + db
    s = max(abs(theta), abs(da), abs(db))
    gamma = s * math.sqrt((theta / s) ** 2 - (da / s) * (db / s))
    if b < a:
        gamma = -gamma
    p = (gamma - da) + theta
    q = ((gamma - da) + gamma) + db
    return a + (p / q) * (b - a)


def _trial_step(stx, fx, dx, sty, fy, dy, stp, fp, dp, brackt, stmin, stmax):
    """One safeguarded trial-step update (the paper's Cases 1-4).

    Returns the updated (stx, fx, dx, sty, fy, dy, stp_new, brackt).
    """
    sgnd = dp * math.copysign(1.0, dx)

    if fp > fx:
        # Case 1: higher function value -- the minimum is bracketed.  Take the
        # cubic step if it is closer to stx than the quadratic step, otherwise
        # the midpoint of the two.
        stpc = _cubic_minimiser(stx, fx, dx, stp, fp, dp)
        stpq = stx + ((dx / ((fx - fp) / (stp - stx) + dx)) / 2.0) * (stp - stx)
        if abs(stpc - stx) < abs(stpq - stx):
            stpf = stpc
        else:
            stpf = stpc + (stpq - stpc) / 2.0
        brackt = True
    elif sgnd < 0.0:
        # Case 2: lower function value, derivatives of opposite sign -- the
        # minimum is bracketed.  Take whichever of the cubic and secant steps
        # lies farther from stp.
        stpc = _cubic_minimiser(stp, fp, dp, stx, fx, dx)
        stpq = stp + (dp / (dp - dx)) * (stx - stp)
        stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
        brackt = True
    elif abs(dp) < abs(dx):
        # Case 3: lower function value, same-sign derivative whose magnitude
        # decreases.  The cubic may have no minimiser in the search direction;
        # then the step goes to the relevant bound.
        theta = 3.0 * (fx - fp) / (stp - stx) + dx + dp
        s = max(abs(theta), abs(dx), abs(dp))
        gamma = s * math.sqrt(max(0.0, (theta / s) ** 2 - (dx / s) * (dp / s)))
        if stp > stx:
            gamma = -gamma
        p = (gamma - dp) + theta
        q = (gamma + (dx - dp)) + gamma
        r = p / q
        if r < 0.0 and gamma != 0.0:
            stpc = stp + r * (stx - stp)
        elif stp > stx:
            stpc = stmax
        else:
            stpc = stmin
        stpq = stp + (dp / (dp - dx)) * (stx - stp)
        if brackt:
            stpf = stpc if abs(stpc - stp) < abs(stpq - stp) else stpq
            limit = stp + _P66 * (sty - stp)
            stpf = min(limit, stpf) if stp > stx else max(limit, stpf)
        else:
            stpf = stpc if abs(stpc - stp) > abs(stpq - stp) else stpq
            stpf = max(stmin, min(stmax, stpf))
    else:
        # Case 4: lower function value, same-sign derivative that does not
        # decrease in magnitude.  Inside a bracket use the cubic through stp
        # and sty; otherwise go to the bound.
        if brackt:
            stpf = _cubic_minimiser(stp, fp, dp, sty, fy, dy)
        elif stp > stx:
            stpf = stmax
        else:
            stpf = stmin

    # Update the interval of uncertainty.
    if fp > fx:
        sty, fy, dy = stp, fp, dp
    else:
        if sgnd < 0.0:
            sty, fy, dy = stx, fx, dx
        stx, fx, dx = stp, fp, dp
    return stx, fx, dx, sty, fy, dy, stpf, brackt


def more_thuente(phi, f0, g0, stp=1.0, ftol=1e-4, gtol=1e-2, xtol=1e-15,
                 stpmin=1e-15, stpmax=1e15, maxfev=20):
    """Search along a descent direction for a strong-Wolfe step.

    ``phi(stp)`` returns (phi(stp), phi'(stp), payload); f0 = phi(0) and
    g0 = phi'(0) < 0 are given.  Returns a LineSearchResult whose status is
    'converged' (both Wolfe conditions hold at ``stp``), or one of 'maxfev',
    'xtol', 'stpmax', 'stpmin', 'rounding' when the search stopped without
    them; ``trials`` lists every evaluated (stp, phi, phi', payload).
    """
    if not (g0 < 0.0):
        raise ValueError("line search needs a descent direction (phi'(0) < 0)")
    if stp <= 0.0:
        raise ValueError("first step must be positive")
    brackt = False
    stage = 1
    gtest = ftol * g0
    width = stpmax - stpmin
    width1 = 2.0 * width
    stx, fx, gx = 0.0, f0, g0
    sty, fy, gy = 0.0, f0, g0
    stmin, stmax = 0.0, stp + _XTRAPU * stp
    trials = []
    nfev = 0
    while True:
        f, g, payload = phi(stp)
        nfev += 1
        trials.append((stp, f, g, payload))
        ftest = f0 + stp * gtest
        if stage == 1 and f <= ftest and g >= 0.0:
            stage = 2
        status = None
        if f <= ftest and abs(g) <= gtol * (-g0):
            status = "converged"
        elif stp == stpmin and (f > ftest or g >= gtest):
            status = "stpmin"
        elif stp == stpmax and f <= ftest and g <= gtest:
            status = "stpmax"
        elif brackt and stmax - stmin <= xtol * stmax:
            status = "xtol"
        elif brackt and (stp <= stmin or stp >= stmax):
            status = "rounding"
        elif nfev >= maxfev:
            status = "maxfev"
        if status is not None:
            return LineSearchResult(stp, f, g, payload, nfev, status, trials)

        if stage == 1 and f <= fx and f > ftest:
            # Work on psi: shift function values by stp*gtest and derivatives
            # by gtest, then shift the interval end values back.
            stx, fxm, gxm, sty, fym, gym, stp, brackt = _trial_step(
                stx, fx - stx * gtest, gx - gtest, sty, fy - sty * gtest, gy - gtest,
                stp, f - stp * gtest, g - gtest, brackt, stmin, stmax)
            fx, gx = fxm + stx * gtest, gxm + gtest
            fy, gy = fym + sty * gtest, gym + gtest
        else:
            stx, fx, gx, sty, fy, gy, stp, brackt = _trial_step(
                stx, fx, gx, sty, fy, gy, stp, f, g, brackt, stmin, stmax)

        if brackt:
            # Force sufficient shrinkage of the bracket, bisecting if needed.
            if abs(sty - stx) >= _P66 * width1:
                stp = stx + 0.5 * (sty - stx)
            width1 = width
            width = abs(sty - stx)
            stmin, stmax = min(stx, sty), max(stx, sty)
        else:
            stmin = stp + _XTRAPL * (stp - stx)
            stmax = stp + _XTRAPU * (stp - stx)
        stp = min(max(stp, stpmin), stpmax)
        if brackt and (stp <= stmin or stp >= stmax or stmax - stmin <= xtol * stmax):
            stp = stx
