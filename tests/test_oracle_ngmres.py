"""Pins of the oracle's N-GMRES Step II and drivers (no GPU)."""
import numpy as np
import pytest

from oracle import cp
from oracle.linesearch import LineSearchResult
from oracle.ngmres import CPProblem, accept_trial, als, ngmres, step2_accelerate
from workloads import initial_guess, test_problem_1, test_problem_2


def test_p7_step2_reproduces_preconditioned_gmres_on_quadratic():
    """Linear case (Section 2.2): N-GMRES without line search and with delta = 0
    gives the GMRES iterate, the minimiser of ||b - A x|| over
    u_0 + K_{i+1}(M^-1 A, M^-1 r_0), here with Jacobi as the one-step process."""
    rng = np.random.default_rng(0)
    n = 30
    Q = rng.standard_normal((n, n))
    A = Q @ Q.T + n * np.eye(n)           # SPD: f = 1/2 x^T A x - b^T x, g = A x - b
    b = rng.standard_normal(n)
    Dinv = 1.0 / np.diag(A)
    M = lambda u: u + Dinv * (b - A @ u)
    g = lambda u: A @ u - b
    u0 = rng.standard_normal(n)
    U, Gw = [u0], [g(u0)]
    r0 = b - A @ u0
    z = Dinv * r0
    for i in range(8):
        u_bar = M(U[-1])
        u_hat, _ = step2_accelerate(np.array(U), np.array(Gw), u_bar, g(u_bar), eps=0.0)
        # explicit Krylov basis of M^-1 A, orthonormalised
        K = [z]
        for _ in range(i):
            K.append(Dinv * (A @ K[-1]))
        Qk, _ = np.linalg.qr(np.array(K).T)
        c = np.linalg.lstsq(A @ Qk, r0, rcond=None)[0]
        x_gmres = u0 + Qk @ c
        assert np.linalg.norm(u_hat - x_gmres) <= 1e-8 * np.linalg.norm(x_gmres)
        U.append(u_hat)
        Gw.append(g(u_hat))


def test_p8_regularised_alpha_matches_lstsq():
    rng = np.random.default_rng(1)
    L, m = 50, 6
    Uw = rng.standard_normal((m, L))
    Gw = rng.standard_normal((m, L))
    u_bar = rng.standard_normal(L)
    g_bar = rng.standard_normal(L)
    _, alpha = step2_accelerate(Uw, Gw, u_bar, g_bar, eps=1e-12)
    P = (g_bar[None, :] - Gw).T
    ref = np.linalg.lstsq(P, -g_bar, rcond=None)[0]
    np.testing.assert_allclose(alpha, ref, rtol=1e-9, atol=1e-9)


def test_r15b_not_positive_definite_gives_alpha_zero():
    """Two window entries with the same gradient and eps = 0: p_1 = p_2 =
    (1, 1, 1, 1), so P^T P = [[4, 4], [4, 4]].  Cholesky: first pivot 4 (root
    2), multiplier 4 / 2 = 2, second pivot 4 - 2 * 2 = 0, not positive: the
    reading takes alpha = 0 and u_hat = u_bar, and flags the step."""
    U = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0]])
    Gw = np.zeros((2, 4))
    u_bar = np.array([5.0, 6.0, 7.0, 8.0])
    g_bar = np.ones(4)
    info = {}
    u_hat, alpha = step2_accelerate(U, Gw, u_bar, g_bar, eps=0.0, info=info)
    assert info["status"] == "not_pd"
    assert np.all(alpha == 0.0) and np.array_equal(u_hat, u_bar)


def test_r15b_regularised_singular_case_by_hand():
    """The same window with eps = 1e-12: delta = 4e-12 makes the matrix
    positive definite; by symmetry alpha_1 = alpha_2 = a with
    (4 + delta) a + 4 a = -4, so a = -4 / (8 + delta), and
    u_hat = u_bar + a (u_bar - u_1) + a (u_bar - u_2)."""
    U = np.array([[0.0, 0.0, 0.0, 0.0], [1.0, 0.0, 0.0, 0.0]])
    Gw = np.zeros((2, 4))
    u_bar = np.array([5.0, 6.0, 7.0, 8.0])
    g_bar = np.ones(4)
    info = {}
    u_hat, alpha = step2_accelerate(U, Gw, u_bar, g_bar, eps=1e-12, info=info)
    a = -4.0 / (8.0 + 4e-12)
    assert info["status"] == "ok"
    np.testing.assert_allclose(alpha, [a, a], rtol=1e-9)
    np.testing.assert_allclose(u_hat, u_bar + a * (2 * u_bar - U[0] - U[1]), rtol=1e-9)


def _ls_result(status, trials):
    last = trials[-1]
    return LineSearchResult(last[0], last[1], last[2], last[3], len(trials), status, trials)


def test_r13_accept_rule_by_hand():
    """Exits without a Wolfe point: the trial with the lowest objective (the
    earliest of equal ones) if it is below f(u_bar) = 3, else beta = 0."""
    g0 = np.array([9.0])
    trials = [(1.0, 5.0, -1.0, "g1"), (0.3, 2.0, -0.5, "g2"), (0.1, 2.5, -0.4, "g3")]
    assert accept_trial(_ls_result("maxfev", trials), 3.0, g0) == (0.3, 2.0, "g2")
    ties = [(1.0, 2.0, -1.0, "g1"), (0.5, 2.0, -0.2, "g2")]
    assert accept_trial(_ls_result("xtol", ties), 3.0, g0) == (1.0, 2.0, "g1")
    worse = [(1.0, 5.0, -1.0, "g1"), (0.5, 3.0, -0.2, "g2")]
    beta, f, g = accept_trial(_ls_result("rounding", worse), 3.0, g0)
    assert beta == 0.0 and f == 3.0 and g is g0
    conv = [(1.0, 5.0, -1.0, "g1"), (0.4, 4.0, 0.0, "g2")]
    assert accept_trial(_ls_result("converged", conv), 3.0, g0) == (0.4, 4.0, "g2")


class _HalvingQuadratic:
    """f(u) = 1/2 ||u||^2 (g = u) with the one-step process M(u) = u / 2 and
    no normalisation: small enough to follow an N-GMRES iteration by hand."""
    R = 1

    def __init__(self):
        self.norm_t, self.nfg = 1.0, 0

    def f_and_g(self, u):
        self.nfg += 1
        return 0.5 * float(u @ u), u.copy()

    def normalise(self, u, g=None):
        return u.copy(), None if g is None else g.copy()

    def als_sweep(self, u, normalise=True):
        return 0.5 * u, []


def test_r13_driver_takes_best_trial_by_hand():
    """u_0 = (2, 0): u_bar = (1, 0), g_bar = (1, 0), p = g_bar - g_0 = (-1, 0),
    alpha = 1 / (1 + 1e-12) (delta = 1e-12), u_hat = (1 - alpha, 0),
    d = (-alpha, 0), slope -alpha.  One trial allowed with a curvature
    tolerance it cannot meet: phi(1) = (1 - alpha)^2 / 2 < f(u_bar) = 1/2, so
    the fallback accepts beta = 1 and u_1 = u_hat."""
    res = ngmres(_HalvingQuadratic(), np.array([2.0, 0.0]), tol=0.0, max_iter=1,
                 ls=dict(maxfev=1, gtol=1e-15))
    r0 = res.trace[0]
    assert r0.ls_status == "maxfev" and r0.nfev == 1 and r0.beta == 1.0 and not r0.restart
    alpha = 1.0 / (1.0 + 1e-12)
    assert abs(res.u[0] - (1.0 - alpha)) <= 1e-15 and res.u[1] == 0.0
    assert abs(res.f - 0.5 * (1.0 - alpha) ** 2) <= 1e-30


def test_r13_driver_falls_back_to_u_bar_by_hand():
    """The same iteration with the first trial at beta = 3: phi(3) =
    (1 - 3 alpha)^2 / 2 ~ 2 > f(u_bar) = 1/2 and no other trial is allowed, so
    beta = 0: u_1 = u_bar = (1, 0), f_1 = 1/2, g_1 = g_bar."""
    res = ngmres(_HalvingQuadratic(), np.array([2.0, 0.0]), tol=0.0, max_iter=1,
                 ls=dict(maxfev=1, gtol=1e-15, stp=3.0))
    r0 = res.trace[0]
    assert r0.ls_status == "maxfev" and r0.beta == 0.0
    assert np.array_equal(res.u, [1.0, 0.0]) and res.f == 0.5
    assert np.array_equal(res.g, [1.0, 0.0])


def test_step2_zero_residual_differences():
    L = 7
    u = np.arange(L, dtype=float)
    g = np.ones(L)
    u_hat, alpha = step2_accelerate(u[None, :] + 1.0, g[None, :], u, g)
    assert np.all(alpha == 0.0) and np.all(u_hat == u)


def _dense_problem(dims, R, c, l1, l2, seed):
    p = test_problem_1(dims, R, c, l1, l2, seed=seed)
    return CPProblem(cp.DenseTensor(p.T), R), p


def test_p10_ngmres_objective_monotone_and_converges():
    prob, _ = _dense_problem((12, 11, 10), 3, 0.9, 1, 1, seed=2)
    u0 = initial_guess((12, 11, 10), 3, seed=10002)
    res = ngmres(prob, u0, tol=1e-9, max_iter=300)
    assert res.converged
    fs = [r.f for r in res.trace]
    half = 0.5 * prob.t.norm2
    assert all(b <= a + 1e-13 * half for a, b in zip(fs, fs[1:]))
    nls = [r for r in res.trace if r.nfev > 0]
    assert len(nls) > 0


def test_p10_als_monotone():
    prob, _ = _dense_problem((10, 9, 8), 3, 0.5, 1, 1, seed=3)
    res = als(prob, initial_guess((10, 9, 8), 3, seed=10003), tol=1e-8, max_iter=400)
    fs = [r.f for r in res.trace]
    half = 0.5 * prob.t.norm2
    assert all(b <= a + 1e-13 * half for a, b in zip(fs, fs[1:]))
    assert res.converged


def _factor_match(A, B):
    """Congruence-based factor match score, best over permutations and signs."""
    import itertools
    R = A[0].shape[1]
    best = 0.0
    for perm in itertools.permutations(range(R)):
        score = 1.0
        for r in range(R):
            s = 1.0
            for a, b in zip(A, B):
                x, y = a[:, r], b[:, perm[r]]
                s *= abs(x @ y) / (np.linalg.norm(x) * np.linalg.norm(y))
            score = min(score, s)
        best = max(best, score)
    return best


def test_p11_exact_recovery_of_noise_free_tensor():
    dims, R = (20, 20, 20), 3
    p = test_problem_1(dims, R, 0.5, 0.0, 0.0, seed=0)
    prob = CPProblem(cp.DenseTensor(p.T), R)
    res = ngmres(prob, initial_guess(dims, R, seed=10000), tol=1e-13, max_iter=500)
    A = cp.split_u(res.u, dims, R)
    rel = cp.objective_direct(p.T, A) / (0.5 * np.sum(p.T ** 2))
    assert rel < 1e-20
    assert _factor_match(A, p.factors) > 1 - 1e-9


def test_sparse_laplacian_ngmres_runs_and_decreases():
    sp = test_problem_2(2, 4)
    prob = CPProblem(cp.CooTensor(sp.dims, sp.coords, sp.values), 3)
    res = ngmres(prob, initial_guess(sp.dims, 3, seed=10011), tol=1e-6, max_iter=200)
    fs = [r.f for r in res.trace]
    assert fs[-1] < fs[0]
    half = 0.5 * prob.t.norm2
    assert all(b <= a + 1e-12 * half for a, b in zip(fs, fs[1:]))


def test_restart_flag_and_window_cap():
    prob, _ = _dense_problem((9, 8, 7), 4, 0.9, 1, 1, seed=4)
    res = ngmres(prob, initial_guess((9, 8, 7), 4, seed=10004), tol=1e-10, max_iter=60, w=3)
    assert all(r.m <= 3 for r in res.trace)
    for a, b in zip(res.trace, res.trace[1:]):
        if a.restart:
            assert b.m == 1


@pytest.mark.slow
def test_p13_ngmres_fewer_iterations_than_als_on_hard_case():
    """Loose behaviour check of Table 3's trend (c = 0.9, high accuracy)."""
    wins = 0
    for seed in range(3):
        prob, _ = _dense_problem((20, 20, 20), 3, 0.9, 0, 0, seed=seed)
        u0 = initial_guess((20, 20, 20), 3, seed=10000 + seed)
        r1 = ngmres(prob, u0, tol=1e-9, max_iter=1500)
        prob2, _ = _dense_problem((20, 20, 20), 3, 0.9, 0, 0, seed=seed)
        r2 = als(prob2, u0, tol=1e-9, max_iter=3000)
        wins += r1.iters < r2.iters
    assert wins >= 2


# ---- steepest descent as the one-step process (N-GMRES preconditioned by SD) ----

class _Quadratic:
    """f(u) = 1/2 u^T A u - b^T u, g = A u - b, no normalisation."""
    R = 1

    def __init__(self, A, b):
        self.A, self.b = A, b
        self.norm_t, self.nfg = 1.0, 0

    def f_and_g(self, u):
        self.nfg += 1
        return 0.5 * float(u @ (self.A @ u)) - float(self.b @ u), self.A @ u - self.b

    def normalise(self, u, g=None):
        return u.copy(), None if g is None else g.copy()


def test_sd_step_unit_gradient_by_hand():
    """f = 1/2 ||u||^2 at u = (0.6, 0.8): g = u, ||g|| = 1, d = -u, so
    phi(beta) = (1 - beta)^2 / 2 and phi'(beta) = -(1 - beta).  The first
    trial beta = 1 is the exact minimiser (phi = phi' = 0, strong Wolfe):
    one evaluation, u_bar = (0, 0), f_bar = 0, g_bar = 0."""
    from oracle.ngmres import sd_step
    prob = _HalvingQuadratic()
    u = np.array([0.6, 0.8])
    u_bar, f_bar, g_bar, nfev = sd_step(prob, u, 0.5, u.copy(), dict(
        stp=1.0, ftol=1e-4, gtol=1e-2, maxfev=20, xtol=1e-15, stpmin=1e-15, stpmax=1e15))
    assert nfev == 1
    assert np.array_equal(u_bar, [0.0, 0.0]) and f_bar == 0.0 and np.array_equal(g_bar, [0.0, 0.0])


def test_sd_step_zero_gradient_leaves_the_iterate():
    from oracle.ngmres import sd_step
    prob = _HalvingQuadratic()
    u = np.array([0.0, 0.0])
    u_bar, f_bar, g_bar, nfev = sd_step(prob, u, 0.0, np.zeros(2), {})
    assert nfev == 0 and prob.nfg == 0 and np.array_equal(u_bar, u) and f_bar == 0.0


def _spd(n, kappa, seed):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.geomspace(1.0, kappa, n)
    return (Q * lam) @ Q.T, rng.standard_normal(n), rng.standard_normal(n)


def test_sd_step_quadratic_within_curvature_bound_of_exact_minimiser():
    """On a quadratic the step is along -g exactly and, with the curvature
    test |phi'(beta)| <= 1e-2 |phi'(0)| met, within 1% of the exact minimiser
    beta* = ||g|| / (d^T A d) along d = -g/||g|| (phi' is linear in beta)."""
    from oracle.ngmres import sd_step
    A, b, u = _spd(20, 50.0, 3)
    prob = _Quadratic(A, b)
    f, g = prob.f_and_g(u)
    ls = dict(stp=1.0, ftol=1e-4, gtol=1e-2, maxfev=20, xtol=1e-15, stpmin=1e-15, stpmax=1e15)
    u_bar, f_bar, g_bar, nfev = sd_step(prob, u, f, g, ls)
    gn = np.linalg.norm(g)
    d = -g / gn
    beta_star = gn / float(d @ (A @ d))
    step = u_bar - u
    beta = float(step @ d)
    assert np.linalg.norm(step - beta * d) <= 1e-12 * np.linalg.norm(step)   # along -g
    assert abs(beta - beta_star) <= 1e-2 * beta_star
    assert f_bar < f and np.allclose(g_bar, A @ u_bar - b, rtol=0, atol=1e-12 * np.linalg.norm(g))
    assert 1 <= nfev <= 20


def test_ngmres_sd_accelerates_steepest_descent_on_quadratic():
    """The preconditioning view (Section 2.2): N-GMRES recombining
    steepest-descent iterates reduces the gradient by 1e6 on an
    ill-conditioned quadratic (kappa = 100) in far fewer iterations than
    steepest descent alone, which has not got there after five times as many
    (48 against 414 iterations here)."""
    from oracle.ngmres import sd_step
    A, b, u0 = _spd(40, 100.0, 4)
    prob = _Quadratic(A, b)
    tol = 1e-6 * np.linalg.norm(A @ u0 - b)
    res = ngmres(prob, u0, tol=tol, max_iter=150, precond="sd")
    assert res.converged
    ls = dict(stp=1.0, ftol=1e-4, gtol=1e-2, maxfev=20, xtol=1e-15, stpmin=1e-15, stpmax=1e15)
    u = u0.copy()
    f, g = prob.f_and_g(u)
    for _ in range(5 * res.iters):
        u, f, g, _ = sd_step(prob, u, f, g, ls)
    assert np.linalg.norm(g) > tol


def test_p10_ngmres_sd_objective_monotone_on_cp_problem():
    """f(u_{i+1}) <= f(u_bar_{i+1}) <= f(u_i): the steepest-descent step and
    the line search of Step III each decrease f or keep the point (R13)."""
    prob, _ = _dense_problem((10, 9, 8), 3, 0.5, 1, 1, seed=5)
    rec = []
    res = ngmres(prob, initial_guess((10, 9, 8), 3, seed=10005), tol=1e-8, max_iter=150,
                 precond="sd", record=rec)
    half = 0.5 * prob.t.norm2
    for r in rec:
        assert r["f_bar"] <= r["f"] + 1e-13 * half
        assert r["f_next"] <= r["f_bar"] + 1e-13 * half
        assert r["nfev_pre"] >= 1
    fs = [r.f for r in res.trace]
    assert fs[-1] < 1e-2 * fs[0] or res.converged
