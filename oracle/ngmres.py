"""FP64 oracle of ALS and N-GMRES for CP decomposition (test infrastructure only).

Follows Section 2 of the paper step by step:

* the one-step process M(u) is one ALS sweep (Section 2.3: nonlinear block
  Gauss-Seidel on G^(n) = 0, n = 1..N, each mode solved with the factors of
  the earlier modes already updated), followed by the normalisation and
  reordering of the rank-one terms;
* one N-GMRES iteration (Section 2.1, Steps I-III and the algorithm box
  "N-GMRES optimization algorithm"): Step I u_bar = M(u_i); Step II the
  accelerated iterate u_hat = u_bar + sum_j alpha_j (u_bar - u_j) over the
  window, with alpha from the regularised normal equations of the linearised
  gradient; Step III a Moré–Thuente line search on f(u_bar + beta (u_hat -
  u_bar)), restart when the direction is not a descent direction, window of
  the last w iterates (Section 2.1 remarks; Section 2.4 parameters).

Readings of points the paper leaves open (shared with the GPU library):
* stopping rule: ||g||_2 / ||T||_F <= tol at the current (normalised) iterate,
  or max_iter iterations;
* restart when g(u_bar)^T d >= 0 (equality counts as non-descent): skip the
  line search, take u_{i+1} = u_bar, and the window restarts from u_{i+1};
* the accelerated iterate u_hat is normalised before d = u_hat - u_bar is
  formed; line-search trial points are not normalised; the accepted iterate
  is normalised and its gradient transformed (not recomputed);
* delta = eps * max diag(P^T P) with eps = 1e-12; if every p_j is zero,
  alpha = 0 (u_hat = u_bar); if P^T P + delta I is still not positive
  definite (a Cholesky pivot that is not positive), alpha = 0 as well and the
  step is flagged;
* if the line search stops without a strong-Wolfe point, the evaluated trial
  with the lowest objective (the earliest of equal ones) is taken when it is
  below f(u_bar), else beta = 0.
"""
from __future__ import annotations

from collections import deque
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg

from . import cp
from .linesearch import more_thuente

__all__ = ["CPProblem", "step2_solve", "step2_accelerate", "accept_trial", "line_search",
           "sd_step", "ngmres_iteration", "ngmres", "als", "IterRecord"]


class CPProblem:
    """f, g and the ALS sweep for a dense or COO data tensor and a rank R."""

    def __init__(self, tensor, R):
        self.t = tensor
        self.R = int(R)
        self.dims = tuple(tensor.dims)
        self.N = len(self.dims)
        self.norm_t = float(np.sqrt(tensor.norm2))
        self.nfg = 0

    def factors(self, u):
        return cp.split_u(u, self.dims, self.R)

    def f_and_g(self, u):
        """Objective (Optimization Problem I) and gradient (Section 2.3)."""
        self.nfg += 1
        A = self.factors(u)
        Ms = [self.t.mttkrp(A, n) for n in range(self.N)]
        G = cp.gradient_from_mttkrps(A, Ms)
        return self.t.objective(A, Ms), cp.join_u(G)

    def normalise(self, u, g=None):
        A = self.factors(u)
        newA, scales, perm = cp.normalise(A)
        u2 = cp.join_u(newA)
        if g is None:
            return u2, None
        G = cp.split_u(g, self.dims, self.R)
        return u2, cp.join_u(cp.transform_gradient(G, scales, perm))

    def als_sweep(self, u, normalise=True):
        """One ALS iteration M(u): solve G^(n) = 0 for A^(n), n = 1..N, in order."""
        A = [a.copy() for a in self.factors(u)]
        flags = []
        for n in range(self.N):
            M = self.t.mttkrp(A, n)
            A[n], flag = cp.mode_solve(M, cp.gamma_bar(A, n))
            flags.append(flag)
        u2 = cp.join_u(A)
        if normalise:
            u2, _ = self.normalise(u2)
        return u2, flags


def step2_solve(P, g_bar, eps=1e-12):
    """alpha of Step II from the rows p_j of P and g_bar.

    Normal equations of the linearised residual ||g_bar + P^T alpha||_2:
    (P P^T + delta I) alpha = -P g_bar with delta = eps * max diag(P P^T)
    (Section 2.1 Step II and fifth remark; Section 2.4).  Returns
    (alpha, status): "ok"; "zero" when every p_j is zero (alpha = 0); "not_pd"
    when the regularised matrix has a Cholesky pivot that is not positive
    (alpha = 0, so u_hat = u_bar).
    """
    B = P @ P.T
    dmax = float(np.max(np.diag(B))) if B.size else 0.0
    if not dmax > 0.0:
        return np.zeros(P.shape[0]), "zero"
    rhs = -(P @ g_bar)
    try:
        c = scipy.linalg.cho_factor(B + eps * dmax * np.eye(B.shape[0]), lower=True)
    except np.linalg.LinAlgError:
        return np.zeros(P.shape[0]), "not_pd"
    return scipy.linalg.cho_solve(c, rhs), "ok"


def step2_accelerate(U, Gw, u_bar, g_bar, eps=1e-12, info=None):
    """N-GMRES Step II: u_hat = u_bar + sum_j alpha_j (u_bar - u_j).

    U, Gw: window iterates and their gradients (m x L); p_j = g_bar - g_j;
    alpha from step2_solve.  If ``info`` is a dict, info["status"] receives
    step2_solve's status.
    """
    U = np.atleast_2d(np.asarray(U, dtype=np.float64))
    Gw = np.atleast_2d(np.asarray(Gw, dtype=np.float64))
    P = g_bar[None, :] - Gw                      # rows are p_j
    alpha, status = step2_solve(P, g_bar, eps)
    if info is not None:
        info["status"] = status
    u_hat = u_bar + np.sum(alpha[:, None] * (u_bar[None, :] - U), axis=0)
    return u_hat, alpha


def accept_trial(res, f0, g0):
    """Step accepted after a line search from (f0, g0) at beta = 0.

    A strong-Wolfe exit takes its own point.  Any other exit takes the
    evaluated trial with the lowest objective (the earliest of equal ones)
    when it is below f0, else beta = 0.  Returns (beta, f, g).
    """
    if res.status == "converged":
        return res.stp, res.f, res.payload
    best = min(res.trials, key=lambda t: t[1])
    if best[1] < f0:
        return best[0], best[1], best[3]
    return 0.0, f0, g0


@dataclass
class IterRecord:
    it: int
    f: float
    rho: float
    beta: float = float("nan")
    restart: bool = False
    nfev: int = 0
    ls_status: str = ""
    m: int = 0
    step2: str = ""


@dataclass
class Result:
    u: np.ndarray
    f: float
    g: np.ndarray
    rho: float
    iters: int
    converged: bool
    trace: list = field(default_factory=list)
    nfg: int = 0


def _rho(problem, g):
    return float(np.linalg.norm(g)) / problem.norm_t


_LS_DEFAULTS = dict(stp=1.0, ftol=1e-4, gtol=1e-2, maxfev=20, xtol=1e-15, stpmin=1e-15,
                   stpmax=1e15)


def line_search(problem, u, f, g, d, slope, ls):
    """Moré–Thuente on phi(beta) = f(u + beta d) from phi(0) = f, phi'(0) =
    slope < 0, then the acceptance rule; returns (beta, f, g, nfev, status)."""
    def phi(beta):
        fb, gb = problem.f_and_g(u + beta * d)
        return fb, float(gb @ d), gb
    res = more_thuente(phi, f, slope, **ls)
    beta, f_new, g_new = accept_trial(res, f, g)
    return beta, f_new, g_new, res.nfev, res.status


def sd_step(problem, u, f, g, ls):
    """Steepest-descent one-step process: u_bar = u + beta d with d = -g/||g||_2
    and beta from the line search (first trial ls["stp"]); u_bar normalised.

    Returns (u_bar, f_bar, g_bar, nfev): f is unchanged by the normalisation
    and the gradient is carried over by its transformation (Section 2.3 end),
    so no further evaluation is needed.  A zero gradient leaves u unchanged.
    """
    gn = float(np.linalg.norm(g))
    if not gn > 0.0:
        return u, f, g, 0
    d = -g / gn
    beta, f_new, g_new, nfev, _ = line_search(problem, u, f, g, d, float(g @ d), ls)
    u_new = u + beta * d if beta != 0.0 else u
    u_bar, g_bar = problem.normalise(u_new, g_new)
    return u_bar, f_new, g_bar, nfev


def ngmres_iteration(problem, u, f, g, U, Gw, eps=1e-12, ls=None, normalise_accel=True,
                     precond="als"):
    """One iteration of the N-GMRES algorithm box from the iterate (u, f, g)
    and the window U, Gw (m x L each, oldest first, ending with u).

    Step I: u_bar = M(u) -- one ALS sweep then f, g at u_bar (precond "als",
    the paper's choice), or the steepest-descent process (precond "sd").
    Step II: u_hat over the window (step2_accelerate), normalised.  Step III:
    restart when g_bar^T d >= 0, else the line search along d = u_hat - u_bar.
    The new iterate is normalised and its gradient transformed.  Returns a
    dict of every intermediate and the new (u_next, f_next, g_next).
    """
    ls = _LS_DEFAULTS | (ls or {})
    out = {}
    if precond == "als":
        u_bar, _ = problem.als_sweep(u)
        f_bar, g_bar = problem.f_and_g(u_bar)
        out["nfev_pre"] = 0
    elif precond == "sd":
        u_bar, f_bar, g_bar, out["nfev_pre"] = sd_step(problem, u, f, g, ls)
    else:
        raise ValueError(f"unknown one-step process {precond!r}")
    s2 = {}
    u_hat, _ = step2_accelerate(U, Gw, u_bar, g_bar, eps, info=s2)
    if normalise_accel:
        u_hat, _ = problem.normalise(u_hat)
    d = u_hat - u_bar
    slope = float(g_bar @ d)
    out.update(u_bar=u_bar, f_bar=f_bar, g_bar=g_bar, u_hat=u_hat, d=d, slope=slope,
               step2=s2["status"], beta=float("nan"), nfev=0, ls_status="")
    if not (slope < 0.0):
        # restart: no line search, the window starts again from the new iterate
        out["restart"] = True
        u_new, f_new, g_new = u_bar, f_bar, g_bar
    else:
        out["restart"] = False
        beta, f_new, g_new, nfev, status = line_search(problem, u_bar, f_bar, g_bar, d, slope, ls)
        out.update(beta=beta, nfev=nfev, ls_status=status)
        u_new = u_bar + beta * d if beta != 0.0 else u_bar
    u_next, g_next = problem.normalise(u_new, g_new)
    out.update(u_next=u_next, f_next=f_new, g_next=g_next)
    return out


def ngmres(problem, u0, tol, max_iter=1000, w=20, eps=1e-12, ls=None,
           normalise_accel=True, record=None, precond="als"):
    """Algorithm "N-GMRES optimization algorithm" with the window grown from 1 to w.

    If ``record`` is a list, one dict per iteration is appended: the state it
    started from (it, u, g, f and the window U, G, oldest first) and every
    value ngmres_iteration returned.
    """
    u, _ = problem.normalise(np.asarray(u0, dtype=np.float64))
    f, g = problem.f_and_g(u)
    window = deque([(u, g)])
    trace = []
    it = 0
    while True:
        rho = _rho(problem, g)
        rec = IterRecord(it=it, f=f, rho=rho, m=len(window))
        trace.append(rec)
        if rho <= tol or it >= max_iter:
            break
        U = np.array([p[0] for p in window])
        Gw = np.array([p[1] for p in window])
        out = ngmres_iteration(problem, u, f, g, U, Gw, eps, ls, normalise_accel, precond)
        rec.step2, rec.restart = out["step2"], out["restart"]
        rec.beta, rec.nfev, rec.ls_status = out["beta"], out["nfev"], out["ls_status"]
        if record is not None:
            record.append(dict(it=it, u=u, g=g, f=f, U=U, G=Gw) | out)
        if out["restart"]:
            window.clear()
        u, f, g = out["u_next"], out["f_next"], out["g_next"]
        window.append((u, g))
        while len(window) > w:
            window.popleft()
        it += 1
    return Result(u=u, f=f, g=g, rho=trace[-1].rho, iters=it,
                  converged=trace[-1].rho <= tol, trace=trace, nfg=problem.nfg)


def als(problem, u0, tol, max_iter=1000):
    """Stand-alone ALS: u_{i+1} = M(u_i), stopped on the same gradient criterion."""
    u, _ = problem.normalise(np.asarray(u0, dtype=np.float64))
    f, g = problem.f_and_g(u)
    trace = []
    it = 0
    while True:
        rho = _rho(problem, g)
        trace.append(IterRecord(it=it, f=f, rho=rho))
        if rho <= tol or it >= max_iter:
            break
        u, _ = problem.als_sweep(u)
        f, g = problem.f_and_g(u)
        it += 1
    return Result(u=u, f=f, g=g, rho=trace[-1].rho, iters=it,
                  converged=trace[-1].rho <= tol, trace=trace, nfg=problem.nfg)
