"""Seeded synthetic inputs shaped like the paper's test problems.

This module only draws inputs.  It holds none of the decomposition method's
arithmetic (no MTTKRP, Gram, gradient, ALS, normalisation or N-GMRES step):
both the CPU oracle and the GPU path receive the arrays produced here and
compute everything else on their own.

Generators
----------
* ``test_problem_1``  -- dense Test Problem I (Section 3): factor matrices
  with prescribed column congruence c, a rank-R canonical tensor built from
  them, then homoscedastic (level l1) and heteroscedastic (level l2) noise,
  generalised from 3-way s x s x s to any order and mode sizes.
* ``test_problem_2``  -- sparse Test Problem II (Section 4): the standard
  finite-difference Laplacian on an s^d grid seen as a 2d-way sparse tensor
  (value 2d on the diagonal, -1 for each grid neighbour, Dirichlet boundary).
* ``sparse_random_cp`` -- large sparse COO tensor with uniformly random
  coordinates whose values are a rank-R canonical tensor sampled at those
  coordinates plus noise (a scale stand-in: the paper's sparse tensors are
  small Laplacians).
* ``random_coo``      -- small random COO tensors for parity tests.
* ``initial_guess``   -- uniformly random U[0,1) factor entries (Section 2.4:
  all initial guesses are uniformly random and shared between methods).
* ``serving_stream``  -- a Poisson stream of decomposition requests of uneven
  order, size and rank.

Conventions: dense tensors are C-order arrays of shape (I_1, ..., I_N) (last
index fastest); a factor A^(n) is an I_n x R array; the iterate u is the
concatenation of the row-major factors.  Seeds drive numpy's PCG64
``default_rng``.
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

__all__ = [
    "congruence_matrix", "collinear_factors", "test_problem_1", "test_problem_2",
    "sparse_random_cp", "random_coo", "initial_guess", "serving_stream",
    "DenseProblem", "SparseProblem", "Request", "noise_scale",
]


def noise_scale(level_percent: float) -> float:
    """Noise-to-signal factor (100/l - 1)^(-1/2) of Test Problem I (Section 3).

    A level of 0 means no noise (the limit of the formula as l -> 0).
    """
    if level_percent <= 0.0:
        return 0.0
    return (100.0 / level_percent - 1.0) ** -0.5


def congruence_matrix(R: int, c: float) -> np.ndarray:
    """R x R matrix with unit diagonal and constant off-diagonal c (Section 3)."""
    K = np.full((R, R), float(c))
    np.fill_diagonal(K, 1.0)
    return K


def collinear_factors(rng: np.random.Generator, dims, R: int, c: float):
    """Factor matrices whose columns have pairwise congruence c (Section 3).

    Each A^(n) is drawn N(0,1), its columns orthonormalised by QR and the
    result multiplied on the right by the upper Cholesky factor U of
    K = U^T U, so that A^(n)^T A^(n) = K exactly.  For a mode with fewer rows
    than R no orthonormal basis exists; there A^(n) = (Z / sqrt(I_n)) U, whose
    Gram matrix equals K in expectation.
    """
    U = np.linalg.cholesky(congruence_matrix(R, c)).T  # upper, K = U^T U
    out = []
    for I in dims:
        Z = rng.standard_normal((I, R))
        if I >= R:
            Q, _ = np.linalg.qr(Z)
            out.append(Q @ U)
        else:
            out.append((Z / math.sqrt(I)) @ U)
    return out


def _full_cp(factors) -> np.ndarray:
    """Dense C-order tensor sum_r a_r^(1) o ... o a_r^(N) (input recipe only)."""
    N = len(factors)
    R = factors[0].shape[1]
    dims = [A.shape[0] for A in factors]
    split = N // 2 if N > 1 else 1
    # rows: C-order index of modes [0, split), columns: modes [split, N)
    left = np.ones((1, R))
    for A in factors[:split]:
        left = (left[:, None, :] * A[None, :, :]).reshape(-1, R)
    right = np.ones((1, R))
    for A in factors[split:]:
        right = (right[:, None, :] * A[None, :, :]).reshape(-1, R)
    return (left @ right.T).reshape(dims)


@dataclass
class DenseProblem:
    T: np.ndarray            # the data tensor (float64 or float32), C-order
    factors: list            # generating factors (float64)
    T_clean: np.ndarray | None = None


def test_problem_1(dims, R: int, c: float, l1: float = 1.0, l2: float = 1.0,
                   seed: int = 0, dtype=np.float64, keep_clean: bool = False) -> DenseProblem:
    """Dense Test Problem I (Section 3), for any order N = len(dims).

    Draw order from ``default_rng(seed)``: the factors of modes 1..N, then the
    noise tensor N1, then N2.  T_hat = T_R + nu(l1) ||T_R|| N1/||N1|| and
    T = T_hat + nu(l2) ||T_hat|| (N2 * T_hat)/||N2 * T_hat|| with
    nu(l) = (100/l - 1)^(-1/2).  The tensor is built in float64 and rounded
    once to ``dtype``; that rounded array is the problem every path solves.
    """
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    factors = collinear_factors(rng, dims, R, c)
    T = _full_cp(factors)
    clean = T.copy() if keep_clean else None
    s1 = noise_scale(l1)
    if s1 > 0.0:
        N1 = rng.standard_normal(dims)
        T += (s1 * np.linalg.norm(T.ravel()) / np.linalg.norm(N1.ravel())) * N1
        del N1
    s2 = noise_scale(l2)
    if s2 > 0.0:
        N2 = rng.standard_normal(dims)
        N2 *= T
        T += (s2 * np.linalg.norm(T.ravel()) / np.linalg.norm(N2.ravel())) * N2
        del N2
    if np.dtype(dtype) != np.float64:
        T = T.astype(dtype)
    return DenseProblem(T=T, factors=factors, T_clean=clean)


@dataclass
class SparseProblem:
    dims: tuple
    coords: np.ndarray   # int32, shape (N, nnz), zero-based
    values: np.ndarray   # float64 or float32, shape (nnz,)


def test_problem_2(d: int, s: int, dtype=np.float64) -> SparseProblem:
    """Sparse Test Problem II (Section 4): the s^d-grid Laplacian as a 2d-way tensor.

    Entry t(x, y) with grid points x = (x_1..x_d), y = (y_1..y_d) (mode order
    x_1..x_d, y_1..y_d) is 2d when y = x and -1 when y is a grid neighbour of
    x; neighbours that fall outside the grid are dropped.  Coordinates are
    listed point by point in C order of x, diagonal first, then the
    neighbours in order of direction k and sign -/+.
    """
    pts = np.stack(np.unravel_index(np.arange(s ** d), (s,) * d), axis=0)  # (d, s^d)
    cols = []
    vals = []
    for p in range(s ** d):
        x = pts[:, p]
        cols.append(np.concatenate([x, x]))
        vals.append(2.0 * d)
        for k in range(d):
            for step in (-1, 1):
                y = x.copy()
                y[k] += step
                if 0 <= y[k] < s:
                    cols.append(np.concatenate([x, y]))
                    vals.append(-1.0)
    coords = np.ascontiguousarray(np.array(cols, dtype=np.int32).T)
    return SparseProblem(dims=(s,) * (2 * d), coords=coords,
                         values=np.array(vals, dtype=dtype))


def sparse_random_cp(dims, nnz_draw: int, R: int, seed: int = 0, l1: float = 1.0,
                     l2: float = 1.0, dtype=np.float32, chunk: int = 1 << 21) -> SparseProblem:
    """Uniform random COO coordinates with values from a rank-R canonical tensor.

    ``nnz_draw`` coordinate tuples are drawn uniformly (int32, one mode after
    the other) from ``default_rng(seed)``; repeated tuples are removed keeping
    the first occurrence, in draw order.  The factors are then drawn N(0,1)
    (I_n x R, modes in order); the values are sum_r prod_n A^(n)(i_n, r) at the
    kept coordinates, plus noise with the Test Problem I formulas applied to
    the value vector (levels l1, l2).  Built in float64, rounded once to dtype.
    """
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    coords = np.stack([rng.integers(0, I, size=nnz_draw, dtype=np.int32) for I in dims])
    key = np.zeros(nnz_draw, dtype=np.int64)
    for n, I in enumerate(dims):
        key = key * I + coords[n].astype(np.int64)
    _, first = np.unique(key, return_index=True)
    del key
    first.sort()
    coords = np.ascontiguousarray(coords[:, first])
    nnz = coords.shape[1]
    factors = [rng.standard_normal((I, R)) for I in dims]
    vals = np.empty(nnz, dtype=np.float64)
    for z0 in range(0, nnz, chunk):
        z1 = min(nnz, z0 + chunk)
        prod = np.ones((z1 - z0, R))
        for n in range(len(dims)):
            prod *= factors[n][coords[n, z0:z1]]
        vals[z0:z1] = prod.sum(axis=1)
    s1 = noise_scale(l1)
    if s1 > 0.0:
        n1 = rng.standard_normal(nnz)
        vals += (s1 * np.linalg.norm(vals) / np.linalg.norm(n1)) * n1
    s2 = noise_scale(l2)
    if s2 > 0.0:
        n2 = rng.standard_normal(nnz) * vals
        vals += (s2 * np.linalg.norm(vals) / np.linalg.norm(n2)) * n2
    return SparseProblem(dims=dims, coords=coords, values=vals.astype(dtype))


def random_coo(dims, nnz: int, seed: int = 0, dtype=np.float64, skew: float = 0.0) -> SparseProblem:
    """Small random COO tensor without duplicates, for parity tests.

    With ``skew`` > 0 the first-mode coordinates follow a power law so that
    some rows hold many nonzeros and many rows hold none (ragged segments).
    """
    dims = tuple(int(d) for d in dims)
    rng = np.random.default_rng(seed)
    total = int(np.prod(dims))
    nnz = min(nnz, total)
    if skew > 0.0:
        w = (np.arange(1, total + 1, dtype=np.float64)) ** (-skew)
        w /= w.sum()
        lin = rng.choice(total, size=nnz, replace=False, p=w)
    else:
        lin = rng.choice(total, size=nnz, replace=False)
    coords = np.stack(np.unravel_index(lin, dims)).astype(np.int32)
    vals = rng.standard_normal(nnz)
    return SparseProblem(dims=dims, coords=np.ascontiguousarray(coords), values=vals.astype(dtype))


def initial_guess(dims, R: int, seed: int) -> np.ndarray:
    """Uniformly random U[0,1) iterate u (all factors, mode order, row-major).

    Section 2.4: initial guesses are uniformly random, and compared methods
    share the same one.  Drawn from ``default_rng(seed)``.
    """
    rng = np.random.default_rng(seed)
    return rng.random(int(sum(dims)) * int(R))


@dataclass
class Request:
    rid: int
    arrival: float       # seconds from stream start
    dims: tuple
    R: int
    c: float
    seed: int


def serving_stream(n_requests: int, rate_per_s: float, seed: int = 7, orders=(3, 4),
                   size_range=(16, 160), rank_range=(2, 24), c_range=(0.0, 0.9)):
    """Poisson stream of decomposition requests of uneven order, size and rank.

    Inter-arrival times are exponential with mean 1/rate; the order is drawn
    from ``orders`` with equal probability, each mode size uniformly from the
    integers in ``size_range``, the rank uniformly from ``rank_range`` and the
    congruence uniformly from ``c_range``.  Request k's tensor seed is 1000 + k.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for k in range(n_requests):
        t += rng.exponential(1.0 / rate_per_s)
        N = int(rng.choice(orders))
        dims = tuple(int(x) for x in rng.integers(size_range[0], size_range[1] + 1, size=N))
        R = int(rng.integers(rank_range[0], rank_range[1] + 1))
        c = float(rng.uniform(*c_range))
        out.append(Request(rid=k, arrival=t, dims=dims, R=R, c=c, seed=1000 + k))
    return out


# These are generators, not tests: keep pytest from collecting them when a
# test module imports them by name.
test_problem_1.__test__ = False
test_problem_2.__test__ = False


def test_problem_1_torch(dims, R: int, c: float, l1: float = 1.0, l2: float = 1.0, seed: int = 0,
                         device="cuda", out_dtype=None):
    """Test Problem I built with torch on a device (for the serving stream).

    The same recipe as ``test_problem_1`` (factors N(0,1) -> QR -> times the
    upper Cholesky factor of the congruence matrix; homoscedastic then
    heteroscedastic noise at levels l1, l2; built in float64, rounded once),
    drawn from a ``torch.Generator(device).manual_seed(seed)`` stream, so the
    values differ from the numpy generator's for the same seed.  Returns the
    flat C-order tensor on the device.
    """
    import torch

    out_dtype = out_dtype or torch.float32
    dims = tuple(int(d) for d in dims)
    g = torch.Generator(device=device)
    g.manual_seed(int(seed))
    K = torch.full((R, R), float(c), dtype=torch.float64, device=device)
    K.fill_diagonal_(1.0)
    U = torch.linalg.cholesky(K).T
    factors = []
    for I in dims:
        Z = torch.randn((I, R), generator=g, dtype=torch.float64, device=device)
        if I >= R:
            Q, _ = torch.linalg.qr(Z)
            factors.append(Q @ U)
        else:
            factors.append((Z / math.sqrt(I)) @ U)
    split = max(1, len(dims) // 2)
    left = torch.ones((1, R), dtype=torch.float64, device=device)
    for A in factors[:split]:
        left = (left[:, None, :] * A[None, :, :]).reshape(-1, R)
    right = torch.ones((1, R), dtype=torch.float64, device=device)
    for A in factors[split:]:
        right = (right[:, None, :] * A[None, :, :]).reshape(-1, R)
    T = (left @ right.T).reshape(-1)
    del left, right
    s1 = noise_scale(l1)
    if s1 > 0.0:
        N1 = torch.randn(T.shape, generator=g, dtype=torch.float64, device=device)
        T += (s1 * torch.linalg.vector_norm(T) / torch.linalg.vector_norm(N1)) * N1
        del N1
    s2 = noise_scale(l2)
    if s2 > 0.0:
        N2 = torch.randn(T.shape, generator=g, dtype=torch.float64, device=device)
        N2 *= T
        T += (s2 * torch.linalg.vector_norm(T) / torch.linalg.vector_norm(N2)) * N2
        del N2
    return T.to(out_dtype)


test_problem_1_torch.__test__ = False
