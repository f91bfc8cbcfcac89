"""Pins of the oracle's N-GMRES Step II and drivers (no GPU)."""
import numpy as np
import pytest

from oracle import cp
from oracle.ngmres import CPProblem, als, ngmres, step2_accelerate
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
