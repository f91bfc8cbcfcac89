"""FP64 oracle of the nonlinear conjugate gradient comparison method (test
infrastructure only).

The paper compares N-GMRES with N-CG using the Polak-Ribiere update and the
same Moré–Thuente line search and parameters (Section 2.4: sufficient-decrease
constant 1e-4, curvature constant 1e-2, first step 1, 20 evaluations).  The
iteration, in the paper's notation for the iterate u and gradient g:

    d_0 = -g_0;  u_{i+1} = u_i + beta_i d_i  (beta_i from the line search on
    phi(beta) = f(u_i + beta d_i));
    gamma_{i+1} = max(0, g_{i+1}^T (g_{i+1} - g_i) / (g_i^T g_i));
    d_{i+1} = -g_{i+1} + gamma_{i+1} d_i.

Readings of points the paper leaves open (shared with the GPU library):
* the Polak-Ribiere coefficient is clipped at zero (the "PR+" form), which
  restarts with steepest descent when it would be negative;
* if a direction is not a descent direction (g^T d >= 0), it is replaced by
  -g before the line search (recorded as a restart);
* the initial guess is normalised like for the other methods; the iterates
  are not (a rescaling of the rank-one terms would break the conjugacy of the
  directions);
* a line search that stops without a strong-Wolfe point takes the evaluated
  trial with the lowest objective if it is below f(u_i), else beta = 0; the
  next direction is then -g (restart);
* stopping: ||g||_2 / ||T||_F <= tol or max_iter, as for N-GMRES.
"""
from __future__ import annotations

import numpy as np

from .linesearch import more_thuente
from .ngmres import IterRecord, Result, _rho, accept_trial

__all__ = ["ncg"]


def ncg(problem, u0, tol, max_iter=1000, ls=None):
    ls = dict(stp=1.0, ftol=1e-4, gtol=1e-2, maxfev=20, xtol=1e-15,
              stpmin=1e-15, stpmax=1e15) | (ls or {})
    u, _ = problem.normalise(np.asarray(u0, dtype=np.float64))
    f, g = problem.f_and_g(u)
    d = -g
    trace = []
    it = 0
    while True:
        rho = _rho(problem, g)
        rec = IterRecord(it=it, f=f, rho=rho)
        trace.append(rec)
        if rho <= tol or it >= max_iter:
            break
        slope = float(g @ d)
        if not (slope < 0.0):
            rec.restart = True
            d = -g
            slope = float(g @ d)

        def phi(beta):
            fb, gb = problem.f_and_g(u + beta * d)
            return fb, float(gb @ d), gb
        res = more_thuente(phi, f, slope, **ls)
        rec.nfev, rec.ls_status = res.nfev, res.status
        beta, f_new, g_new = accept_trial(res, f, g)
        restart_next = res.status != "converged"
        rec.beta = beta
        u_new = u + beta * d if beta != 0.0 else u
        if restart_next:
            d = -g_new
        else:
            gamma = max(0.0, float(g_new @ (g_new - g)) / float(g @ g))
            d = -g_new + gamma * d
        u, f, g = u_new, f_new, g_new
        it += 1
    return Result(u=u, f=f, g=g, rho=trace[-1].rho, iters=it,
                  converged=trace[-1].rho <= tol, trace=trace, nfg=problem.nfg)
