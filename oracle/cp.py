"""FP64 oracle of the CP tensor quantities (test infrastructure only).

Parity pins: tests/test_oracle_cp.py.

Notation follows the paper: an N-way tensor T of size I_1 x ... x I_N, a
canonical rank-R tensor [[A^(1), ..., A^(N)]] (Section 1, definition of A_R),
factor matrices A^(n) of size I_n x R, the iterate u = all factor entries
stacked (mode order, each factor row-major).

Dense tensors are numpy arrays in C order.  Sparse tensors are coordinate
lists: ``coords`` (N x nnz, zero-based ints) and ``values`` (nnz,).
"""
from __future__ import annotations

import numpy as np
import scipy.linalg

__all__ = [
    "split_u", "join_u", "matricize", "khatri_rao", "mttkrp", "mttkrp_coo",
    "grams", "gamma", "gamma_bar", "full_tensor", "objective_direct",
    "objective_identity", "gradient_from_mttkrps", "normalise",
    "transform_gradient", "mode_solve", "DenseTensor", "CooTensor",
]


# ---------------------------------------------------------------- iterate ---

def split_u(u, dims, R):
    """Factor matrices A^(n) (I_n x R views) from the stacked iterate u."""
    out, off = [], 0
    for I in dims:
        out.append(np.asarray(u[off:off + I * R], dtype=np.float64).reshape(I, R))
        off += I * R
    if off != len(u):
        raise ValueError("iterate length does not match dims and R")
    return out


def join_u(factors):
    """Stacked iterate u from factor matrices (mode order, row-major)."""
    return np.concatenate([np.asarray(A, dtype=np.float64).ravel() for A in factors])


# ------------------------------------------------------------------ MTTKRP ---

def matricize(T, n):
    """Mode-n matricisation T_(n) (Section 2.3): I_n x prod_{l != n} I_l.

    Columns enumerate the remaining indices in C order (last mode fastest);
    this is the column order that pairs with ``khatri_rao`` below.
    """
    T = np.asarray(T, dtype=np.float64)
    return np.moveaxis(T, n, 0).reshape(T.shape[n], -1)


def khatri_rao(mats):
    """Column-wise Kronecker product A_1 (.) A_2 (.) ... (.) A_k.

    Row index is the C-order linear index of (i_1, ..., i_k), last fastest,
    so row (i_1..i_k) holds prod_j A_j(i_j, r) (Section 2.3, definition of Phi).
    """
    R = mats[0].shape[1]
    out = np.ones((1, R))
    for A in mats:
        out = (out[:, None, :] * np.asarray(A, dtype=np.float64)[None, :, :]).reshape(-1, R)
    return out


def mttkrp(T, factors, n):
    """M^(n) = T_(n) Phibar^(n)  (Section 2.3, gradient formula and Phi definitions).

    Element form: M^(n)(i, r) = sum over all indices with i_n = i of
    T(i_1..i_N) prod_{k != n} A^(k)(i_k, r).  Written as the explicit
    matricisation times the explicit Khatri-Rao product of the other factors.
    """
    others = [factors[k] for k in range(len(factors)) if k != n]
    if not others:   # order 1: the empty Khatri-Rao product is a row of ones
        return matricize(T, n) @ np.ones((1, factors[n].shape[1]))
    return matricize(T, n) @ khatri_rao(others)


def mttkrp_coo(dims, coords, values, factors, n):
    """Sparse MTTKRP by the element definition summed over the nonzeros.

    M^(n)(i, r) = sum_{z : i_n(z) = i} v_z prod_{k != n} A^(k)(i_k(z), r).
    """
    R = factors[0].shape[1]
    v = np.asarray(values, dtype=np.float64)
    contrib = v[:, None] * np.ones((len(v), R))
    for k in range(len(dims)):
        if k != n:
            contrib = contrib * factors[k][np.asarray(coords[k], dtype=np.int64)]
    M = np.zeros((dims[n], R))
    np.add.at(M, np.asarray(coords[n], dtype=np.int64), contrib)
    return M


# ------------------------------------------------------- Grams and Gamma ---

def grams(factors):
    """S^(k) = A^(k)^T A^(k) for every mode k (Section 2.3, Gamma definitions)."""
    return [A.T @ A for A in factors]


def gamma(factors):
    """Gamma = Hadamard product of all S^(k) (Section 2.3)."""
    G = np.ones((factors[0].shape[1],) * 2)
    for S in grams(factors):
        G = G * S
    return G


def gamma_bar(factors, n):
    """Gammabar^(n) = Hadamard product of S^(k) over k != n (Section 2.3)."""
    G = np.ones((factors[0].shape[1],) * 2)
    for k, S in enumerate(grams(factors)):
        if k != n:
            G = G * S
    return G


# ------------------------------------------------------ objective / grad ---

def full_tensor(factors):
    """[[A^(1)..A^(N)]] = sum_r a_r^(1) o ... o a_r^(N)  (Section 1), term by term."""
    dims = tuple(A.shape[0] for A in factors)
    R = factors[0].shape[1]
    out = np.zeros(dims)
    for r in range(R):
        term = np.array(1.0)
        for A in factors:
            term = np.multiply.outer(term, A[:, r])
        out += term
    return out


def objective_direct(T, factors):
    """f = 1/2 ||T - [[A]]||_F^2  (Section 1, Optimization Problem I), by the residual."""
    D = np.asarray(T, dtype=np.float64) - full_tensor(factors)
    return 0.5 * float(np.sum(D * D))


def objective_identity(norm_t2, factors, M, n):
    """f from the expansion 1/2||T||^2 - <T,[[A]]> + 1/2||[[A]]||^2.

    <T,[[A]]> = sum_{i,r} A^(n)(i,r) M^(n)(i,r) for any mode n, and
    ||[[A]]||^2 = sum_{r,s} Gamma(r,s)  (follows from the definitions of
    Section 1 and Section 2.3; not printed in the paper).
    """
    return 0.5 * norm_t2 - float(np.sum(factors[n] * M)) + 0.5 * float(np.sum(gamma(factors)))


def gradient_from_mttkrps(factors, Ms):
    """G^(n) = -M^(n) + A^(n) Gammabar^(n)  (Section 2.3, gradient formula)."""
    return [-Ms[n] + factors[n] @ gamma_bar(factors, n) for n in range(len(factors))]


# ---------------------------------------------------------- normalisation ---

def normalise(factors):
    """Normalise and reorder the rank-one terms (Section 2.3, last paragraph).

    For each term r: nu_r^(n) = ||a_r^(n)||_2, lambda_r = prod_n nu_r^(n); every
    factor vector becomes unit length times lambda_r^(1/N), i.e. is scaled by
    s_r^(n) = lambda_r^(1/N) / nu_r^(n); terms are then ordered by decreasing
    lambda_r (stable: equal lambdas keep their original order).  A term with a
    zero column has lambda_r = 0: all its columns become zero (scale 0) and it
    sorts last.

    Returns (new_factors, scales (N x R, before permutation), perm) with
    new_factors[n][:, j] = scales[n, perm[j]] * factors[n][:, perm[j]].
    """
    N = len(factors)
    R = factors[0].shape[1]
    nu = np.array([np.sqrt(np.sum(A * A, axis=0)) for A in factors])  # N x R
    lam = np.prod(nu, axis=0)
    root = lam ** (1.0 / N)
    scales = np.zeros((N, R))
    for n in range(N):
        for r in range(R):
            scales[n, r] = root[r] / nu[n, r] if lam[r] > 0.0 else 0.0
    perm = np.argsort(-lam, kind="stable")
    new = [(factors[n] * scales[n][None, :])[:, perm] for n in range(N)]
    return new, scales, perm


def transform_gradient(G, scales, perm):
    """Gradient at the normalised point from the gradient before normalising.

    f is unchanged when term r's columns are scaled by s_r^(n) with
    prod_n s_r^(n) = 1, so dF/d(s a) = (dF/da) / s: column r of G^(n) is
    divided by s_r^(n) and then permuted like the factors.  Columns with a
    zero scale (vanished terms) are left undivided.
    """
    out = []
    for n, Gn in enumerate(G):
        s = scales[n].copy()
        s[s == 0.0] = 1.0
        out.append((Gn / s[None, :])[:, perm])
    return out


# -------------------------------------------------------------- ALS solve ---

def mode_solve(M, Gbar):
    """Solve A Gammabar = M for A (the optimality equation G^(n) = 0, Section 2.3).

    Cholesky of the symmetric Gammabar^(n) (scipy).  If it is not positive
    definite: retry with Gammabar + 1e-14 tr(Gammabar)/R I, then fall back to
    the pseudo-inverse from a symmetric eigendecomposition.  Returns
    (A, flag) with flag 0 = Cholesky, 1 = shifted Cholesky, 2 = pseudo-inverse.
    """
    R = Gbar.shape[0]
    try:
        c = scipy.linalg.cho_factor(Gbar, lower=True, check_finite=True)
        return scipy.linalg.cho_solve(c, M.T).T, 0
    except np.linalg.LinAlgError:
        pass
    shift = 1e-14 * np.trace(Gbar) / R
    try:
        c = scipy.linalg.cho_factor(Gbar + shift * np.eye(R), lower=True)
        return scipy.linalg.cho_solve(c, M.T).T, 1
    except np.linalg.LinAlgError:
        w, V = np.linalg.eigh(Gbar)
        tol = R * np.finfo(float).eps * max(abs(w).max(), 1e-300)
        winv = np.where(abs(w) > tol, 1.0 / np.where(w == 0, 1.0, w), 0.0)
        return M @ (V * winv[None, :]) @ V.T, 2


# ------------------------------------------------------- tensor wrappers ---

class DenseTensor:
    """Dense data tensor (float64 view of the given array).

    objective="direct" (default) evaluates f by the residual; "identity" by
    the expansion through the last mode's MTTKRP and Gamma, the form a fast
    path uses (used to gauge how much the choice of formula alone moves a
    result near convergence).
    """

    def __init__(self, T, objective="direct"):
        self.T = np.asarray(T, dtype=np.float64)
        self.dims = self.T.shape
        self.norm2 = float(np.sum(self.T * self.T))
        if objective not in ("direct", "identity"):
            raise ValueError(objective)
        self.form = objective

    def mttkrp(self, factors, n):
        return mttkrp(self.T, factors, n)

    def objective(self, factors, Ms=None):
        if self.form == "identity" and Ms is not None:
            n = len(self.dims) - 1
            return objective_identity(self.norm2, factors, Ms[n], n)
        return objective_direct(self.T, factors)


class CooTensor:
    """Sparse coordinate-format data tensor (no duplicate coordinates)."""

    def __init__(self, dims, coords, values):
        self.dims = tuple(int(d) for d in dims)
        self.coords = np.asarray(coords, dtype=np.int64)
        self.values = np.asarray(values, dtype=np.float64)
        self.norm2 = float(np.sum(self.values * self.values))

    def mttkrp(self, factors, n):
        return mttkrp_coo(self.dims, self.coords, self.values, factors, n)

    def objective(self, factors, Ms):
        n = len(self.dims) - 1
        return objective_identity(self.norm2, factors, Ms[n], n)

    def to_dense(self):
        T = np.zeros(self.dims)
        np.add.at(T, tuple(self.coords), self.values)
        return T
