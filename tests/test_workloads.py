"""Pins of the seeded generators (P12): invariants the paper's recipes fix."""
import os

import numpy as np
import pytest
import scipy.sparse as sps

from workloads import (collinear_factors, congruence_matrix, initial_guess, noise_scale,
                       random_coo, serving_stream, sparse_random_cp, test_problem_1,
                       test_problem_2)

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("dims,R,c", [((20, 20, 20), 3, 0.5), ((30, 17, 25, 9), 5, 0.9),
                                      ((6, 40), 8, 0.0)])
def test_factor_gram_is_congruence_matrix(dims, R, c):
    A = collinear_factors(np.random.default_rng(0), dims, R, c)
    K = congruence_matrix(R, c)
    for a in A:
        if a.shape[0] >= R:          # exact only where an orthonormal basis exists
            np.testing.assert_allclose(a.T @ a, K, rtol=0, atol=1e-14)
        else:
            assert a.shape == (a.shape[0], R) and np.all(np.isfinite(a))


def test_noise_levels_follow_formula():
    p = test_problem_1((10, 11, 12), 3, 0.5, l1=1.0, l2=5.0, seed=4, keep_clean=True)
    rng = np.random.default_rng(4)
    collinear_factors(rng, (10, 11, 12), 3, 0.5)
    N1 = rng.standard_normal((10, 11, 12))
    T_hat = p.T_clean + noise_scale(1.0) * np.linalg.norm(p.T_clean) / np.linalg.norm(N1) * N1
    assert abs(np.linalg.norm(T_hat - p.T_clean) / np.linalg.norm(p.T_clean)
               - (100 / 1.0 - 1) ** -0.5) < 1e-12
    assert abs(np.linalg.norm(p.T - T_hat) / np.linalg.norm(T_hat) - (100 / 5.0 - 1) ** -0.5) < 1e-12
    assert noise_scale(0.0) == 0.0


def test_float32_tensor_is_single_rounding():
    p64 = test_problem_1((9, 8, 7), 2, 0.5, seed=5)
    p32 = test_problem_1((9, 8, 7), 2, 0.5, seed=5, dtype=np.float32)
    assert p32.T.dtype == np.float32
    np.testing.assert_array_equal(p32.T, p64.T.astype(np.float32))


def _laplacian_matrix(d, s):
    L1 = sps.diags([-np.ones(s - 1), 2 * np.ones(s), -np.ones(s - 1)], [-1, 0, 1])
    out = sps.csr_matrix((s ** d, s ** d))
    for k in range(d):
        mats = [sps.identity(s)] * d
        mats[k] = L1
        term = mats[0]
        for m in mats[1:]:
            term = sps.kron(term, m)
        out = out + term
    return out.toarray()


@pytest.mark.parametrize("d,s", [(1, 5), (2, 4), (3, 3), (2, 6)])
def test_tp2_equals_kron_sum_laplacian(d, s):
    sp = test_problem_2(d, s)
    N = 2 * d
    assert sp.coords.shape == (N, s ** d + 2 * d * s ** (d - 1) * (s - 1))
    T = np.zeros(sp.dims)
    T[tuple(sp.coords)] = sp.values
    np.testing.assert_array_equal(T.reshape(s ** d, s ** d), _laplacian_matrix(d, s))


def test_tp2_nnz_for_paper_instance():
    assert test_problem_2(3, 6).coords.shape[1] == 1296


def test_tp2_golden_fixtures():
    ref = np.loadtxt(os.path.join(GOLDEN, "tp2_d1_s4.txt"))
    sp = test_problem_2(1, 4)
    T = np.zeros(sp.dims)
    T[tuple(sp.coords)] = sp.values
    np.testing.assert_array_equal(T, ref)
    ent = np.loadtxt(os.path.join(GOLDEN, "tp2_d2_s3_entries.txt"))
    sp = test_problem_2(2, 3)
    T = np.zeros(sp.dims)
    T[tuple(sp.coords)] = sp.values
    R = np.zeros((3, 3, 3, 3))
    for row in ent:
        R[tuple(int(x) for x in row[:4])] = row[4]
    np.testing.assert_array_equal(T, R)


def test_sparse_random_cp_no_duplicates_and_values():
    sp = sparse_random_cp((50, 60, 70), 5000, 4, seed=1, l1=0, l2=0, dtype=np.float64)
    key = sp.coords[0].astype(np.int64) * 4200 + sp.coords[1].astype(np.int64) * 70 + sp.coords[2]
    assert len(np.unique(key)) == sp.coords.shape[1]
    rng = np.random.default_rng(1)
    for I in (50, 60, 70):
        rng.integers(0, I, size=5000, dtype=np.int32)
    F = [rng.standard_normal((I, 4)) for I in (50, 60, 70)]
    z = 17
    i, j, k = sp.coords[:, z]
    assert abs(sp.values[z] - np.sum(F[0][i] * F[1][j] * F[2][k])) < 1e-12


def test_random_coo_and_stream_shapes():
    sp = random_coo((5, 6, 7), 100, seed=2, skew=1.5)
    assert sp.coords.shape == (3, 100)
    reqs = serving_stream(50, 10.0, seed=1)
    assert all(16 <= d <= 160 for r in reqs for d in r.dims)
    assert all(2 <= r.R <= 24 and len(r.dims) in (3, 4) for r in reqs)
    assert all(b.arrival > a.arrival for a, b in zip(reqs, reqs[1:]))
    u = initial_guess((3, 4), 2, seed=1)
    assert u.shape == (14,) and np.all((u >= 0) & (u < 1))
