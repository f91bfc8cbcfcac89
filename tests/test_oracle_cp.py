"""Pins of the FP64 oracle's tensor quantities against brute force, closed forms
and library routines (no GPU).  Each test is labelled with its pin number (P1,
P2, ...) in the project's list of oracle pins."""
import itertools

import numpy as np
import pytest

from oracle import cp
from workloads import random_coo, test_problem_1

rng0 = np.random.default_rng(12345)


def _rand_factors(dims, R, seed):
    rng = np.random.default_rng(seed)
    return [rng.standard_normal((I, R)) for I in dims]


def _brute_mttkrp(T, factors, n):
    """M^(n)(i,r) = sum over all index tuples with i_n = i of T * prod_{k!=n} A^(k)."""
    dims = T.shape
    R = factors[0].shape[1]
    M = np.zeros((dims[n], R))
    for idx in itertools.product(*[range(d) for d in dims]):
        for r in range(R):
            p = T[idx]
            for k in range(len(dims)):
                if k != n:
                    p *= factors[k][idx[k], r]
            M[idx[n], r] += p
    return M


def _brute_full(factors):
    dims = tuple(A.shape[0] for A in factors)
    R = factors[0].shape[1]
    X = np.zeros(dims)
    for idx in itertools.product(*[range(d) for d in dims]):
        X[idx] = sum(np.prod([factors[k][idx[k], r] for k in range(len(dims))]) for r in range(R))
    return X


@pytest.mark.parametrize("dims", [(3, 4, 5), (2, 3, 2, 3), (4, 1, 3), (2, 2, 2, 2, 2), (6,), (3, 4)])
@pytest.mark.parametrize("R", [1, 2, 4])
def test_p1_mttkrp_matches_brute_force(dims, R):
    T = np.random.default_rng(1).standard_normal(dims)
    A = _rand_factors(dims, R, 2)
    for n in range(len(dims)):
        M = cp.mttkrp(T, A, n)
        Mb = _brute_mttkrp(T, A, n)
        assert np.max(np.abs(M - Mb)) <= 1e-14 * max(1.0, np.max(np.abs(Mb)))


@pytest.mark.parametrize("dims,R", [((5, 6, 7), 3), ((3, 4, 2, 5), 4)])
def test_p1_inner_product_same_for_every_mode(dims, R):
    T = np.random.default_rng(3).standard_normal(dims)
    A = _rand_factors(dims, R, 4)
    ref = float(np.sum(T * _brute_full(A)))
    for n in range(len(dims)):
        val = float(np.sum(A[n] * cp.mttkrp(T, A, n)))
        assert abs(val - ref) <= 1e-12 * max(1.0, abs(ref))


def test_p1_planted_mistake_is_caught():
    """A transposed Khatri-Rao order (first factor fastest) fails the brute force."""
    dims, R = (3, 4, 5), 2
    T = np.random.default_rng(5).standard_normal(dims)
    A = _rand_factors(dims, R, 6)
    wrong = cp.matricize(T, 0) @ cp.khatri_rao([A[2], A[1]])
    assert np.max(np.abs(wrong - _brute_mttkrp(T, A, 0))) > 1e-3


@pytest.mark.parametrize("dims,nnz,R", [((4, 5, 6), 40, 3), ((3, 3, 4, 2), 30, 2), ((7, 2, 5), 70, 5)])
def test_p2_coo_mttkrp_matches_dense(dims, nnz, R):
    sp = random_coo(dims, nnz, seed=7)
    A = _rand_factors(dims, R, 8)
    T = np.zeros(dims)
    for z in range(sp.coords.shape[1]):
        T[tuple(sp.coords[:, z])] = sp.values[z]
    for n in range(len(dims)):
        Ms = cp.mttkrp_coo(dims, sp.coords, sp.values, A, n)
        Md = _brute_mttkrp(T, A, n)
        assert np.max(np.abs(Ms - Md)) <= 1e-13 * max(1.0, np.max(np.abs(Md)))


def test_p3_gamma_sum_is_norm_of_canonical_tensor():
    dims, R = (4, 3, 5, 2), 3
    A = _rand_factors(dims, R, 9)
    X = _brute_full(A)
    np.testing.assert_allclose(cp.full_tensor(A), X, rtol=0, atol=1e-13)
    assert abs(np.sum(cp.gamma(A)) - np.sum(X * X)) <= 1e-12 * np.sum(X * X)
    for n in range(len(dims)):
        Gb = cp.gamma_bar(A, n)
        # Gammabar^(n) is the Gram matrix of the Khatri-Rao product of the others
        KR = cp.khatri_rao([A[k] for k in range(len(dims)) if k != n])
        np.testing.assert_allclose(Gb, KR.T @ KR, rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("dims,R", [((4, 5, 3), 2), ((3, 2, 4, 3), 3)])
def test_p4_gradient_matches_finite_differences(dims, R):
    rng = np.random.default_rng(10)
    T = rng.standard_normal(dims)
    A = _rand_factors(dims, R, 11)
    u = cp.join_u(A)
    Ms = [cp.mttkrp(T, A, n) for n in range(len(dims))]
    g = cp.join_u(cp.gradient_from_mttkrps(A, Ms))
    f = lambda v: cp.objective_direct(T, cp.split_u(v, dims, R))
    for trial in range(5):
        d = rng.standard_normal(u.size)
        h = 1e-5
        fd = (f(u + h * d) - f(u - h * d)) / (2 * h)
        an = float(g @ d)
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an))


def test_p4_gradient_vanishes_at_exact_decomposition():
    dims, R = (5, 6, 4), 3
    A = _rand_factors(dims, R, 12)
    T = _brute_full(A)
    Ms = [cp.mttkrp(T, A, n) for n in range(3)]
    g = cp.join_u(cp.gradient_from_mttkrps(A, Ms))
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(T)


def test_objective_identity_matches_direct_residual():
    dims, R = (4, 5, 6), 3
    T = np.random.default_rng(13).standard_normal(dims)
    A = _rand_factors(dims, R, 14)
    fd = cp.objective_direct(T, A)
    for n in range(3):
        fi = cp.objective_identity(float(np.sum(T * T)), A, cp.mttkrp(T, A, n), n)
        assert abs(fi - fd) <= 1e-12 * np.sum(T * T)


@pytest.mark.parametrize("dims,R", [((4, 5, 6), 3), ((3, 4, 2, 3), 2)])
def test_p5_mode_update_equals_lstsq(dims, R):
    T = np.random.default_rng(15).standard_normal(dims)
    A = _rand_factors(dims, R, 16)
    for n in range(len(dims)):
        KR = cp.khatri_rao([A[k] for k in range(len(dims)) if k != n])
        ref = np.linalg.lstsq(KR, cp.matricize(T, n).T, rcond=None)[0].T
        got, flag = cp.mode_solve(cp.mttkrp(T, A, n), cp.gamma_bar(A, n))
        assert flag == 0
        np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-10)


def test_p6_als_mode_updates_are_monotone():
    prob = test_problem_1((8, 7, 9), 3, 0.9, 1, 1, seed=3)
    T = prob.T
    R = 3
    A = _rand_factors(T.shape, R, 17)
    half = 0.5 * np.sum(T * T)
    f_prev = cp.objective_direct(T, A)
    for sweep in range(5):
        for n in range(3):
            A[n], _ = cp.mode_solve(cp.mttkrp(T, A, n), cp.gamma_bar(A, n))
            f_new = cp.objective_direct(T, A)
            assert f_new <= f_prev + 1e-13 * half
            f_prev = f_new


def test_mode_solve_singular_fallbacks():
    M = np.ones((4, 2))
    Gb = np.array([[1.0, 1.0], [1.0, 1.0]])        # rank one: Cholesky fails
    A, flag = cp.mode_solve(M, Gb)
    assert flag in (1, 2)
    assert np.all(np.isfinite(A))
    # least-squares consistent: A Gb reproduces the projection of M onto range(Gb)
    np.testing.assert_allclose(A @ Gb, M, rtol=1e-6, atol=1e-6)


def test_p14_normalisation_invariants():
    dims, R = (5, 4, 6), 4
    rng = np.random.default_rng(18)
    T = rng.standard_normal(dims)
    A = _rand_factors(dims, R, 19)
    A[1][:, 2] *= 40.0     # make term 2 dominant so the order changes
    B, scales, perm = cp.normalise(A)
    # the canonical tensor is unchanged
    np.testing.assert_allclose(cp.full_tensor(B), cp.full_tensor(A), rtol=0, atol=1e-12)
    # column norms equal across modes, lambdas descending
    nu = np.array([np.linalg.norm(b, axis=0) for b in B])
    np.testing.assert_allclose(nu, np.repeat(nu[:1], 3, axis=0), rtol=1e-13)
    lam = np.prod(nu, axis=0)
    assert np.all(np.diff(lam) <= 0)
    assert perm[0] == 2
    # transformed gradient equals the gradient recomputed at the new point
    G = cp.gradient_from_mttkrps(A, [cp.mttkrp(T, A, n) for n in range(3)])
    Gt = cp.transform_gradient(G, scales, perm)
    Gr = cp.gradient_from_mttkrps(B, [cp.mttkrp(T, B, n) for n in range(3)])
    for a, b in zip(Gt, Gr):
        np.testing.assert_allclose(a, b, rtol=1e-10, atol=1e-10)


def test_normalisation_zero_term_and_ties():
    A = [np.array([[1.0, 0.0, 2.0], [0.0, 0.0, 0.0]]),
         np.array([[1.0, 3.0, 1.0], [1.0, 0.0, 1.0]])]
    B, scales, perm = cp.normalise(A)
    # term 1 has a zero column: lambda 0, sorted last, columns all zero
    assert perm[-1] == 1
    assert np.all(B[0][:, -1] == 0) and np.all(B[1][:, -1] == 0)
    # terms 0 and 2: lambdas 1*sqrt2 and 2*sqrt2 -> term 2 first
    assert list(perm[:2]) == [2, 0]
    # equal lambdas keep original order (stable)
    C = [np.eye(3), np.eye(3)]
    _, _, p2 = cp.normalise(C)
    assert list(p2) == [0, 1, 2]
