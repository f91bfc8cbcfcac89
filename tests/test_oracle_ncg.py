"""Pins of the oracle's N-CG comparison method (Section 2.4: Polak-Ribiere
update, the same Moré–Thuente line search), no GPU."""
import numpy as np
import pytest

from oracle import cp as ocp
from oracle.ncg import ncg
from oracle.ngmres import CPProblem
from workloads import initial_guess, test_problem_1


class Quadratic:
    """f = 1/2 u^T A u - b^T u (A SPD), g = A u - b; no normalisation."""

    def __init__(self, A, b):
        self.A, self.b = A, b
        self.norm_t = 1.0
        self.nfg = 0

    def f_and_g(self, u):
        self.nfg += 1
        Au = self.A @ u
        return 0.5 * float(u @ Au) - float(self.b @ u), Au - self.b

    def normalise(self, u, g=None):
        return u, g


def _linear_cg(A, b, x0, iters):
    """Textbook linear conjugate gradients (closed-form step and coefficient)."""
    x = x0.copy()
    r = b - A @ x
    p = r.copy()
    xs = [x.copy()]
    for _ in range(iters):
        Ap = A @ p
        alpha = float(r @ r) / float(p @ Ap)
        x = x + alpha * p
        r_new = r - alpha * Ap
        p = r_new + (float(r_new @ r_new) / float(r @ r)) * p
        r = r_new
        xs.append(x.copy())
    return xs


def test_ncg_on_a_quadratic_is_linear_cg():
    """With a (near) exact line search, Polak-Ribiere equals Fletcher-Reeves on
    a quadratic and N-CG reproduces linear CG iterate by iterate; it finishes
    in at most n steps."""
    rng = np.random.default_rng(3)
    n = 12
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + 0.5 * np.eye(n)
    b = rng.standard_normal(n)
    x0 = rng.standard_normal(n)
    prob = Quadratic(A, b)
    res = ncg(prob, x0, tol=0.0, max_iter=8, ls=dict(gtol=1e-12, xtol=1e-18))
    # the objective sequence of the first 8 iterates is linear CG's
    xs = _linear_cg(A, b, x0, 8)
    fl = [0.5 * float(x @ A @ x) - float(b @ x) for x in xs]
    fo = [r.f for r in res.trace]
    np.testing.assert_allclose(fo, fl, rtol=1e-9, atol=1e-9 * abs(fl[0]))
    # n steps take the gradient down by ~6 orders (from there the line search
    # works on objective differences at rounding level, the stall of N-CG
    # near the solution that the paper describes for its CP runs)
    full = ncg(Quadratic(A, b), x0, tol=0.0, max_iter=n + 1, ls=dict(gtol=1e-12, xtol=1e-18))
    assert full.trace[n + 1].rho <= 1e-6 * full.trace[0].rho


def test_ncg_first_step_is_steepest_descent():
    rng = np.random.default_rng(4)
    n = 6
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + np.eye(n)
    b = rng.standard_normal(n)
    x0 = np.zeros(n)
    res = ncg(Quadratic(A, b), x0, tol=0.0, max_iter=1, ls=dict(gtol=1e-12, xtol=1e-18))
    # exact minimiser along -g0 = b from 0: x1 = (b.b / b.A.b) b
    x1 = (float(b @ b) / float(b @ A @ b)) * b
    assert abs(res.trace[0].beta - float(b @ b) / float(b @ A @ b)) <= 1e-9 * abs(res.trace[0].beta)
    np.testing.assert_allclose(res.u, x1, rtol=1e-9, atol=1e-12)


def test_ncg_on_cp_decreases_f_and_converges():
    dims, R = (12, 11, 10), 3
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=2)
    prob = CPProblem(ocp.DenseTensor(p.T), R)
    res = ncg(prob, initial_guess(dims, R, seed=10002), tol=1e-6, max_iter=600)
    f = [r.f for r in res.trace]
    assert all(b <= a + 1e-13 * f[0] for a, b in zip(f, f[1:]))   # sufficient decrease or beta = 0
    assert res.converged


def test_ncg_objective_decreases_on_a_quadratic():
    """Every accepted step satisfies sufficient decrease; no restart is needed
    on a convex quadratic (the PR coefficient stays a descent direction)."""
    rng = np.random.default_rng(5)
    n = 5
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + np.eye(n)
    b = rng.standard_normal(n)
    res = ncg(Quadratic(A, b), rng.standard_normal(n), tol=0.0, max_iter=4,
              ls=dict(gtol=1e-12, xtol=1e-18))
    f = [r.f for r in res.trace]
    assert all(b2 < a for a, b2 in zip(f, f[1:]))
    assert not any(r.restart for r in res.trace)
