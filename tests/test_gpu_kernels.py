"""GPU parity of the hot-path building blocks against the FP64 oracle.

Every call goes through the C ABI (libcpng.so) via the ctypes binding; the
expected values come only from ``oracle``.  Inputs are seeded and synthetic
(``workloads``), at sizes that span several workgroup tiles with ragged tails.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cp as ocp
from oracle.ngmres import step2_accelerate
from workloads import random_coo, test_problem_1, test_problem_2

from helpers import TOL, abs_mttkrp, abs_mttkrp_coo, assert_close_to_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_1105_5331_amd as cpng
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    with cpng.Handle(0) as handle:
        yield handle


def _cpng():
    import paper_1105_5331_amd as cpng
    return cpng


def _dev(x, dtype=None):
    t = torch.from_numpy(np.ascontiguousarray(x))
    if dtype is not None:
        t = t.to(dtype)
    return t.cuda()


def _factors(dims, R, seed, scale=1.0):
    rng = np.random.default_rng(seed)
    return [scale * rng.standard_normal((I, R)) for I in dims]


# Generic-kernel shapes (ragged, odd sizes) and shapes whose inner modes are
# multiples of 8, which take the streaming MFMA kernels in BF16X3 mode (partial
# last K-step, several row chunks, order 2 and 5).
DENSE_SHAPES = [(3, 4, 5), (20, 20, 20), (33, 17, 45), (7, 9, 5, 11), (70, 3, 130),
                (2, 3, 2, 3, 2), (2, 2, 3, 2, 2, 3, 2, 2), (1, 65, 1, 3), (129, 2, 67),
                (9, 40, 32), (130, 7, 24, 16), (64, 64, 64), (17, 136), (24, 8), (300, 16, 8),
                (5, 6, 7, 8, 16), (7,), (40, 36), (13, 12)]


@pytest.mark.parametrize("dims", DENSE_SHAPES)
@pytest.mark.parametrize("R", [1, 3, 10, 17, 33])
@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp32in_fp64acc"])
def test_dense_mttkrp_parity(h, dims, R, prec):
    cpng = _cpng()
    print(f"case dense mttkrp dims={dims} R={R} prec={prec}", flush=True)
    rng = np.random.default_rng(abs(hash((dims, R))) % 2**32)
    T64 = rng.standard_normal(dims)
    if prec == "fp64":
        T = T64
        Tt = _dev(T)
    else:
        T = T64.astype(np.float32)
        Tt = _dev(T)
    A = _factors(dims, R, 5)
    u = _dev(ocp.join_u(A))
    Tg = cpng.Tensor(dims, Tt.reshape(-1))
    for n in range(len(dims)):
        M = cpng.cp_mttkrp(h, Tg, u, R, n, prec).cpu().numpy()
        ref = ocp.mttkrp(T.astype(np.float64), A, n)
        bound = abs_mttkrp(T.astype(np.float64), A, n)
        assert_close_to_bound(M, ref, bound, TOL[prec], f"mode {n}")
        if prec == "bf16x3":
            assert np.linalg.norm(M - ref) <= 1e-3 * max(np.linalg.norm(ref), 1e-300)


def test_dense_mttkrp_bitwise_repeatable(h):
    cpng = _cpng()
    dims, R = (40, 50, 60), 16
    T = np.random.default_rng(1).standard_normal(dims).astype(np.float32)
    u = _dev(ocp.join_u(_factors(dims, R, 2)))
    Tg = cpng.Tensor(dims, _dev(T).reshape(-1))
    for prec in ("fp32", "bf16x3", "fp64"):
        for n in range(3):
            a = cpng.cp_mttkrp(h, Tg, u, R, n, prec).cpu().numpy()
            b = cpng.cp_mttkrp(h, Tg, u, R, n, prec).cpu().numpy()
            assert np.array_equal(a, b)


def test_mttkrp_argument_errors(h):
    cpng = _cpng()
    dims, R = (4, 5, 6), 3
    T64 = _dev(np.ones(dims))
    Tg = cpng.Tensor(dims, T64.reshape(-1))
    u = _dev(np.ones(15 * R))
    with pytest.raises(cpng.CpError) as e:
        cpng.cp_mttkrp(h, Tg, u, R, 3, "fp64")
    assert e.value.code == -1
    with pytest.raises(cpng.CpError):
        cpng.cp_mttkrp(h, Tg, u, R, 0, "fp32")     # fp32 needs a float32 tensor
    with pytest.raises(cpng.CpError):
        cpng.cp_mttkrp(h, Tg, u, 0, 0, "fp64")


@pytest.mark.parametrize("dims,R", [((5, 300, 7), 4), ((20, 20, 20, 3), 33), ((1, 1, 2), 1),
                                    ((130, 3, 64), 64), ((5000, 3000, 10), 16)])
def test_gram_parity(h, dims, R):
    cpng = _cpng()
    A = _factors(dims, R, 7)
    S, Gb, G = cpng.cp_gram(h, dims, _dev(ocp.join_u(A)), R)
    S, Gb, G = S.cpu().numpy(), Gb.cpu().numpy(), G.cpu().numpy()
    for k in range(len(dims)):
        ref = A[k].T @ A[k]
        np.testing.assert_allclose(S[k], ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())
        refb = ocp.gamma_bar(A, k)
        np.testing.assert_allclose(Gb[k], refb, rtol=1e-11, atol=1e-12 * np.abs(refb).max())
    refg = ocp.gamma(A)
    np.testing.assert_allclose(G, refg, rtol=1e-11, atol=1e-12 * np.abs(refg).max())


# one-workgroup form (L = R sum_k I_k <= 8192) and, for the larger shapes,
# the multi-block form (rows packed 64 / R to a wave: 1 at R = 40 and 64, 4 at
# R = 16, 6 at R = 10 with four idle lanes)
@pytest.mark.parametrize("dims,R", [((6, 7, 8), 5), ((30, 4, 9, 3), 12), ((3, 2), 1),
                                    ((300, 200, 100), 40), ((3000, 40), 16),
                                    ((701, 499, 3), 10), ((200, 100, 50), 64)])
def test_normalize_parity(h, dims, R):
    cpng = _cpng()
    A = _factors(dims, R, 8)
    A[0][:, R // 2] *= 30.0
    G = _factors(dims, R, 9)
    u, g = _dev(ocp.join_u(A)), _dev(ocp.join_u(G))
    cpng.cp_normalize(h, dims, u, R, g)
    B, scales, perm = ocp.normalise(A)
    Gt = ocp.transform_gradient(G, scales, perm)
    np.testing.assert_allclose(u.cpu().numpy(), ocp.join_u(B), rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(g.cpu().numpy(), ocp.join_u(Gt), rtol=1e-12, atol=1e-14)


@pytest.mark.parametrize("dims,R", [((3, 4), 3), ((3000, 40), 8)])
def test_normalize_zero_term(h, dims, R):
    """A zero term goes last; its gradient columns are left undivided."""
    cpng = _cpng()
    A = _factors(dims, R, 10)
    A[1][:, 0] = 0.0
    G = _factors(dims, R, 11)
    u, g = _dev(ocp.join_u(A)), _dev(ocp.join_u(G))
    cpng.cp_normalize(h, dims, u, R, g)
    B, scales, perm = ocp.normalise(A)
    assert perm[-1] == 0
    np.testing.assert_allclose(u.cpu().numpy(), ocp.join_u(B), rtol=1e-12, atol=1e-14)
    Gt = ocp.transform_gradient(G, scales, perm)
    np.testing.assert_allclose(g.cpu().numpy(), ocp.join_u(Gt), rtol=1e-12, atol=1e-14)


# (5, 2500, 6): the left group's mode 0 sums 2500 pairs per output (split-K
# second level); every other case has short sums (one-launch second level)
@pytest.mark.parametrize("dims,R,c", [((20, 20, 20), 3, 0.5), ((13, 30, 8, 5), 6, 0.9),
                                      ((70, 9, 66), 10, 0.3), ((5, 7, 6, 4, 3), 40, 0.5),
                                      ((130, 3, 70), 64, 0.2), ((3, 90), 7, 0.4),
                                      ((5, 2500, 6), 3, 0.5)])
@pytest.mark.parametrize("prec", ["fp64", "fp32in_fp64acc"])
def test_objective_grad_parity(h, dims, R, c, prec):
    """All N MTTKRPs at one point (dense order >= 3: the two mode-group
    partials, then each mode from its group's partial) and the gradient
    epilogue, float64 accumulation, against the oracle on the same (float64 or
    float32) tensor."""
    cpng = _cpng()
    print(f"case objective_grad dims={dims} R={R} prec={prec}", flush=True)
    dt = np.float64 if prec == "fp64" else np.float32
    p = test_problem_1(dims, R, c, 1, 1, seed=3, dtype=dt)
    T64 = p.T.astype(np.float64)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    half = 0.5 * np.sum(T64 ** 2)
    assert abs(Tg.norm_sq - 2 * half) <= 1e-12 * 2 * half
    A = _factors(dims, R, 11, scale=0.5)
    f, g = cpng.cp_objective_grad(h, Tg, _dev(ocp.join_u(A)), R, prec)
    fo = ocp.objective_direct(T64, A)
    go = ocp.join_u(ocp.gradient_from_mttkrps(A, [ocp.mttkrp(T64, A, n) for n in range(len(dims))]))
    assert abs(f.item() - fo) <= 1e-12 * half
    assert np.linalg.norm(g.cpu().numpy() - go) <= 1e-12 * np.sqrt(2 * half)


@pytest.mark.parametrize("prec,tol", [("fp32", 1e-5), ("bf16x3", 1e-4)])
def test_objective_grad_reduced_precision(h, prec, tol):
    """Per-iterate tolerance of the reduced-precision bulk (same input u):
    |df| / (1/2 ||T||^2) and ||dg|| / ||T|| against the FP64 oracle."""
    cpng = _cpng()
    dims, R = (40, 36, 44), 8
    p = test_problem_1(dims, R, 0.9, 1, 1, seed=4, dtype=np.float32)
    T64 = p.T.astype(np.float64)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    A = _factors(dims, R, 12, scale=0.5)
    f, g = cpng.cp_objective_grad(h, Tg, _dev(ocp.join_u(A)), R, prec)
    half = 0.5 * np.sum(T64 ** 2)
    fo = ocp.objective_direct(T64, A)
    go = ocp.join_u(ocp.gradient_from_mttkrps(A, [ocp.mttkrp(T64, A, n) for n in range(3)]))
    assert abs(f.item() - fo) / half <= tol
    assert np.linalg.norm(g.cpu().numpy() - go) / np.sqrt(2 * half) <= tol


# split points: (33, 21, 40) s=2; (12, 7, 9, 24) s=2, both groups two modes;
# (130, 3, 64) s=1, one-mode left group, inner length 130 (generic kernel for
# the right partial); (5, 300, 8) s=2; (4, 6, 5, 8, 3) s=3, uncovered inner lengths.
@pytest.mark.parametrize("dims,R", [((33, 21, 40), 17), ((9, 10, 16), 40), ((12, 7, 9, 24), 5),
                                    ((130, 3, 64), 32), ((5, 300, 8), 1), ((4, 6, 5, 8, 3), 9)])
def test_objective_grad_bf16x3_two_level(h, dims, R):
    """BF16x3 bulk through the two group partials (each a BF16x3 MTTKRP of
    the reshaped tensor) and the float64 second level: the per-iterate
    tolerance of the BF16x3 path."""
    cpng = _cpng()
    print(f"case objective_grad bf16x3 two-level dims={dims} R={R}", flush=True)
    p = test_problem_1(dims, R, 0.7, 1, 1, seed=6, dtype=np.float32)
    T64 = p.T.astype(np.float64)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    A = _factors(dims, R, 14, scale=0.5)
    f, g = cpng.cp_objective_grad(h, Tg, _dev(ocp.join_u(A)), R, "bf16x3")
    half = 0.5 * np.sum(T64 ** 2)
    fo = ocp.objective_direct(T64, A)
    go = ocp.join_u(ocp.gradient_from_mttkrps(A, [ocp.mttkrp(T64, A, n) for n in range(len(dims))]))
    assert abs(f.item() - fo) / (half + abs(fo)) <= 1e-4
    assert np.linalg.norm(g.cpu().numpy() - go) / (np.sqrt(2 * half) + np.linalg.norm(go)) <= 1e-4


@pytest.mark.parametrize("dims,R,c,prec", [((20, 20, 20), 3, 0.5, "fp64"), ((9, 14, 6, 11), 5, 0.9, "fp64"),
                                           ((33, 70, 65), 12, 0.5, "fp32in_fp64acc"),
                                           ((6, 5, 7, 4, 6), 36, 0.3, "fp64"),
                                           ((17, 9, 32), 20, 0.5, "bf16x3"),
                                           ((300, 12, 10), 8, 0.5, "fp64")])
def test_als_sweep_parity(h, dims, R, c, prec):
    """One ALS sweep (every mode's MTTKRP from its group's partial, the right
    group's formed after the left modes' updates) against the oracle's
    sequential sweep."""
    cpng = _cpng()
    from oracle.ngmres import CPProblem
    print(f"case als_sweep dims={dims} R={R} prec={prec}", flush=True)
    p = test_problem_1(dims, R, c, 1, 1, seed=5, dtype=np.float64 if prec == "fp64" else np.float32)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    A = _factors(dims, R, 13)
    u = _dev(ocp.join_u(A))
    cpng.cp_als_sweep(h, Tg, u, R, prec, normalize=True)
    prob = CPProblem(ocp.DenseTensor(p.T.astype(np.float64)), R)
    ref, flags = prob.als_sweep(ocp.join_u(A))
    assert flags == [0] * len(dims)
    if prec == "bf16x3":   # ~1e-6 MTTKRP error, amplified by the mode solves
        np.testing.assert_allclose(u.cpu().numpy(), ref, rtol=1e-3, atol=1e-4)
    else:
        np.testing.assert_allclose(u.cpu().numpy(), ref, rtol=1e-9, atol=1e-11)


def test_als_sweep_zero_term_takes_shifted_cholesky(h):
    """A zero column in A^(2) makes Gammabar^(1) exactly singular (zero row and
    column): both sides fail plain Cholesky on that exact zero pivot and take
    the shifted factorisation; the zero term stays zero."""
    cpng = _cpng()
    from oracle.ngmres import CPProblem
    dims, R = (6, 5, 4), 3
    A = _factors(dims, R, 14)
    A[2][:, 1] = 0.0
    T = np.random.default_rng(15).standard_normal(dims)
    Tg = cpng.Tensor(dims, _dev(T).reshape(-1))
    u = _dev(ocp.join_u(A))
    cpng.cp_als_sweep(h, Tg, u, R, "fp64", normalize=False)
    prob = CPProblem(ocp.DenseTensor(T), R)
    ref, flags = prob.als_sweep(ocp.join_u(A), normalise=False)
    assert flags[0] == 1
    got = u.cpu().numpy()
    np.testing.assert_allclose(got, ref, rtol=1e-9, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("case", ["spd", "zero_row", "indefinite", "rank_one_exact"])
def test_mode_solve_paths(h, case):
    """cp_mode_solve takes the oracle's path (Cholesky / shifted / pseudo-inverse)
    on matrices where the path is decided exactly, and gives the same A."""
    cpng = _cpng()
    rng = np.random.default_rng(16)
    R, I = 4, 37
    M = rng.standard_normal((I, R))
    if case == "spd":
        Q = rng.standard_normal((R, R))
        G = Q @ Q.T + R * np.eye(R)
    elif case == "zero_row":
        Q = rng.standard_normal((R, R))
        G = Q @ Q.T + R * np.eye(R)
        G[2, :] = 0.0
        G[:, 2] = 0.0
        M[:, 2] = 0.0
    elif case == "indefinite":
        G = np.array([[0.0, 1.0, 0, 0], [1.0, 0.0, 0, 0], [0, 0, 2.0, 0], [0, 0, 0, -3.0]])
    else:
        G = np.zeros((R, R))
        G[0, 0] = 4.0       # only one nonzero pivot, the rest exactly zero
        M[:, 1:] = 0.0
    A, kind = cpng.cp_mode_solve(h, _dev(M), _dev(G))
    ref, flag = ocp.mode_solve(M, G)
    assert kind == flag
    np.testing.assert_allclose(A.cpu().numpy(), ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("R,case", [(1, "spd"), (16, "spd"), (17, "spd"), (32, "spd"), (33, "spd"),
                                    (64, "spd"), (40, "zero_row"), (24, "zero_row")])
def test_mode_solve_rank_widths(h, R, case):
    """The register Cholesky at every width it is compiled for (R <= 16, 32,
    64) and across the boundaries; a zero row makes it fail at that pivot and
    the shifted factorisation take over, as in the oracle."""
    cpng = _cpng()
    print(f"case mode_solve R={R} {case}", flush=True)
    rng = np.random.default_rng(100 + R)
    I = 53
    M = rng.standard_normal((I, R))
    Q = rng.standard_normal((R, R))
    G = Q @ Q.T + R * np.eye(R)
    if case == "zero_row":
        k = R // 2
        G[k, :] = 0.0
        G[:, k] = 0.0
        M[:, k] = 0.0
    A, kind = cpng.cp_mode_solve(h, _dev(M), _dev(G))
    ref, flag = ocp.mode_solve(M, G)
    assert kind == flag == (0 if case == "spd" else 1)
    np.testing.assert_allclose(A.cpu().numpy(), ref, rtol=1e-10, atol=1e-12)


@pytest.mark.parametrize("L,m", [(1, 1), (1000, 5), (40000, 20), (333, 64)])
def test_ngmres_accelerate_parity(h, L, m):
    cpng = _cpng()
    rng = np.random.default_rng(L + m)
    U = rng.standard_normal((m, L))
    G = rng.standard_normal((m, L))
    ub = rng.standard_normal(L)
    gb = rng.standard_normal(L)
    uh, alpha, _ = cpng.ngmres_accelerate(h, _dev(U), _dev(G), _dev(ub), _dev(gb), 1e-12)
    ref_u, ref_a = step2_accelerate(U, G, ub, gb, 1e-12)
    np.testing.assert_allclose(alpha.cpu().numpy(), ref_a, rtol=1e-8, atol=1e-10)
    np.testing.assert_allclose(uh.cpu().numpy(), ref_u, rtol=1e-8, atol=1e-10)


def test_ngmres_accelerate_zero_differences(h):
    cpng = _cpng()
    L = 50
    g = np.ones(L)
    uh, alpha, _ = cpng.ngmres_accelerate(h, _dev(np.zeros((2, L))), _dev(np.stack([g, g])),
                                       _dev(np.arange(L, dtype=float)), _dev(g))
    assert np.all(alpha.cpu().numpy() == 0.0)
    np.testing.assert_array_equal(uh.cpu().numpy(), np.arange(L, dtype=float))


# ------------------------------------------------------------------ sparse ---

def _sparse(cpng, sp, dtype):
    vals = _dev(sp.values.astype(dtype))
    return cpng.Tensor(sp.dims, vals, coords=_dev(sp.coords))


SPARSE_CASES = [
    ("tp2_d2_s4", lambda: test_problem_2(2, 4)),
    ("tp2_d3_s3", lambda: test_problem_2(3, 3)),
    ("tp2_d4_s3", lambda: test_problem_2(4, 3)),      # order 8, two waves
    ("rand_small", lambda: random_coo((7, 8, 9), 100, seed=1)),
    ("rand_ragged", lambda: random_coo((300, 40, 50), 9000, seed=2, skew=1.2)),
    ("rand_4way", lambda: random_coo((17, 23, 5, 31), 4000, seed=3)),
    ("long_rows", lambda: random_coo((3, 200, 200), 20000, seed=4)),
    # larger modes (thousands of rows), many waves per mode, and with skew
    # very uneven rows
    ("blocked_3way", lambda: random_coo((50, 3000, 40), 30000, seed=5)),
    ("blocked_skew", lambda: random_coo((40, 3000, 30), 6000, seed=6, skew=1.2)),
    ("blocked_4way", lambda: random_coo((2500, 30, 20, 12), 20000, seed=7)),
]


@pytest.mark.parametrize("name,make", SPARSE_CASES)
@pytest.mark.parametrize("prec", ["fp64", "fp32"])
@pytest.mark.parametrize("R", [1, 5, 16, 40])
def test_sparse_mttkrp_parity(h, name, make, prec, R):
    cpng = _cpng()
    print(f"case sparse mttkrp {name} R={R} prec={prec}", flush=True)
    sp = make()
    dtype = np.float64 if prec == "fp64" else np.float32
    vals = sp.values.astype(dtype).astype(np.float64)
    Tg = _sparse(cpng, sp, dtype)
    cpng.cp_tensor_prepare(h, Tg)
    A = _factors(sp.dims, R, 21)
    u = _dev(ocp.join_u(A))
    for n in range(len(sp.dims)):
        M = cpng.cp_mttkrp(h, Tg, u, R, n, prec).cpu().numpy()
        ref = ocp.mttkrp_coo(sp.dims, sp.coords, vals, A, n)
        bound = abs_mttkrp_coo(sp.dims, sp.coords, vals, A, n)
        assert_close_to_bound(M, ref, bound, TOL[prec], f"{name} mode {n}")
    cpng.cp_tensor_release(h, Tg)


def test_sparse_empty_and_errors(h):
    cpng = _cpng()
    dims = (4, 5, 6)
    T = cpng.Tensor(dims, torch.zeros(0, dtype=torch.float64, device="cuda"),
                    coords=torch.zeros((3, 0), dtype=torch.int32, device="cuda"))
    cpng.cp_tensor_prepare(h, T)
    M = cpng.cp_mttkrp(h, T, _dev(np.ones(15 * 2)), 2, 1, "fp64").cpu().numpy()
    assert np.all(M == 0)
    # duplicate coordinates are rejected
    coords = np.array([[0, 1, 0], [2, 2, 2], [3, 3, 3]], dtype=np.int32)
    Td = cpng.Tensor(dims, _dev(np.ones(3)), coords=_dev(coords))
    with pytest.raises(cpng.CpError) as e:
        cpng.cp_tensor_prepare(h, Td)
    assert e.value.code == -5
    # out-of-range coordinate is rejected
    coords = np.array([[0, 4], [0, 0], [0, 0]], dtype=np.int32)
    Tb = cpng.Tensor(dims, _dev(np.ones(2)), coords=_dev(coords))
    with pytest.raises(cpng.CpError) as e:
        cpng.cp_tensor_prepare(h, Tb)
    assert e.value.code == -1


def test_sparse_objective_grad_parity(h):
    cpng = _cpng()
    sp = random_coo((30, 20, 25), 3000, seed=9, skew=0.8)
    R = 4
    Tg = _sparse(cpng, sp, np.float64)
    cpng.cp_tensor_prepare(h, Tg)
    A = _factors(sp.dims, R, 22, scale=0.7)
    f, g = cpng.cp_objective_grad(h, Tg, _dev(ocp.join_u(A)), R, "fp64")
    t = ocp.CooTensor(sp.dims, sp.coords, sp.values)
    Ms = [t.mttkrp(A, n) for n in range(3)]
    fo = t.objective(A, Ms)
    go = ocp.join_u(ocp.gradient_from_mttkrps(A, Ms))
    half = 0.5 * t.norm2
    assert abs(f.item() - fo) <= 1e-12 * half
    assert np.linalg.norm(g.cpu().numpy() - go) <= 1e-12 * np.sqrt(t.norm2)


def test_profile_select_times_only_the_chosen_kernels(h):
    """With only the dense MTTKRP selected, a two-level objective/gradient
    evaluation records its group-partial launches and no second-level ones;
    an unknown id bit is rejected."""
    cpng = _cpng()
    dims, R = (24, 20, 18, 16), 3
    T = _dev(np.random.default_rng(5).standard_normal(dims).astype(np.float32))
    Tg = cpng.Tensor(dims, T)
    cpng.cp_tensor_prepare(h, Tg)
    u = _dev(ocp.join_u(_factors(dims, R, 23)))
    cpng.cp_profile_select(h, 1 << cpng.CP_KERNEL_DENSE_MTTKRP)
    cpng.cp_profile(h, True)
    cpng.cp_objective_grad(h, Tg, u, R, "fp32")
    torch.cuda.synchronize()
    nd, msd = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_MTTKRP)
    ng, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_GROUP_MTTKRP)
    cpng.cp_profile(h, False)
    cpng.cp_profile_select(h, 0xFF)
    assert nd >= 1 and msd > 0 and ng == 0
    cpng.cp_profile(h, True)
    cpng.cp_objective_grad(h, Tg, u, R, "fp32")
    torch.cuda.synchronize()
    ng, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_GROUP_MTTKRP)
    cpng.cp_profile(h, False)
    assert ng >= 1
    # float64-accumulating precisions are timed under their own id
    cpng.cp_profile(h, True)
    cpng.cp_mttkrp(h, Tg, u, R, 0, "fp32in_fp64acc")
    cpng.cp_mttkrp(h, Tg, u, R, 0, "fp32")
    torch.cuda.synchronize()
    n64, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_MTTKRP_F64)
    n32, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_MTTKRP)
    cpng.cp_profile(h, False)
    assert n64 == 1 and n32 == 1
    with pytest.raises(cpng.CpError):
        cpng.cp_profile_select(h, 1 << 8)


def test_sparse_gather_reference(h):
    """The sparse gather measurement kernel runs on a prepared COO tensor in
    every mode, is timed under its own id, and rejects a dense tensor."""
    cpng = _cpng()
    sp = random_coo((300, 40, 50), 9000, seed=2, dtype=np.float32)
    Tg = cpng.Tensor(sp.dims, _dev(sp.values), _dev(sp.coords))
    cpng.cp_tensor_prepare(h, Tg)
    R = 16
    u = _dev(ocp.join_u(_factors(sp.dims, R, 3)))
    cpng.cp_profile(h, True)
    for n in range(3):
        cpng.cp_sparse_gather_read(h, Tg, u, R, n)
    torch.cuda.synchronize()
    nl, ms = cpng.cp_profile_read(h, cpng.CP_KERNEL_SPARSE_GATHER)
    cpng.cp_profile(h, False)
    assert nl == 3 and ms > 0
    Td = cpng.Tensor((4, 5, 6), _dev(np.ones(120, dtype=np.float32)))
    with pytest.raises(cpng.CpError):
        cpng.cp_sparse_gather_read(h, Td, _dev(np.ones(15 * R)), R, 0)


def test_stream_read_reference(h):
    """The streaming-read measurement kernel: runs on an aligned buffer, is
    timed under its own id, and rejects a misaligned or ragged one."""
    cpng = _cpng()
    x = torch.ones(1 << 20, dtype=torch.float32, device="cuda")
    cpng.cp_profile(h, True)
    cpng.cp_stream_read(h, x)
    torch.cuda.synchronize()
    n, ms = cpng.cp_profile_read(h, cpng.CP_KERNEL_STREAM_READ)
    cpng.cp_profile(h, False)
    assert n == 1 and ms > 0
    with pytest.raises(cpng.CpError):
        cpng.cp_stream_read(h, x[1:])          # 4-byte offset, ragged length
