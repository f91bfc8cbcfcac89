"""Parity at the full benchmark sizes, in the launch configuration bench.py
times, on sampled outputs: whole rows M^(n)(i, :) recomputed by the oracle
from the definition restricted to the sampled indices i.

* dense 128^4 float32, R = 32 (BF16X3 and FP32 kernels, every mode), as
  single-mode MTTKRPs and as the gradient of the two-level evaluation that
  the benchmark step runs (both mode-group partials on the reshaped tensor,
  the float64 second level and the fused epilogue);
* sparse 20000^3 COO with about 2e7 nonzeros, R = 16 (FP32, every mode);
* dense 200^3, R = 10, congruence 0.9 (the time-to-gradient study): f and g
  at the initial guess in every precision, whole (the oracle finishes them
  in about a second).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cp as ocp
from workloads import initial_guess, sparse_random_cp, test_problem_1

from helpers import TOL, assert_close_to_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_1105_5331_amd as cpng
    with cpng.Handle(0) as handle:
        yield handle


def test_dense_128x4_R32_sampled_rows(h):
    import paper_1105_5331_amd as cpng
    dims, R = (128, 128, 128, 128), 32
    print("case dense 128^4 R=32 full size", flush=True)
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=0, dtype=np.float32)
    Tg = cpng.Tensor(dims, torch.from_numpy(p.T).cuda().reshape(-1))
    u0 = initial_guess(dims, R, seed=10000)
    A = ocp.split_u(u0, dims, R)
    u = torch.from_numpy(u0).cuda()
    rows = [0, 77, 127]
    T64 = p.T   # float32; the oracle widens the sampled slices exactly
    for n in range(4):
        sl = np.take(T64, rows, axis=n).astype(np.float64)
        An = [a if k != n else A[n][rows] for k, a in enumerate(A)]
        ref = ocp.mttkrp(sl, An, n)
        bound = ocp.mttkrp(np.abs(sl), [np.abs(a) for a in An], n)
        for prec in ("bf16x3", "fp32"):
            M = cpng.cp_mttkrp(h, Tg, u, R, n, prec).cpu().numpy()[rows]
            assert_close_to_bound(M, ref, bound, TOL[prec], f"mode {n} {prec}")


@pytest.mark.parametrize("prec", ["bf16x3", "fp32", "fp32in_fp64acc"])
def test_dense_128x4_R32_gradient_rows(h, prec):
    """G^(n)(i, :) = -M^(n)(i, :) + A^(n)(i, :) Gammabar^(n) on sampled rows of
    every mode, from cp_objective_grad (the two-level evaluation, both group
    partials from one pass of the two-sided kernel), against the oracle's
    rows; the bound adds |A| |Gammabar| to the MTTKRP bound."""
    import paper_1105_5331_amd as cpng
    dims, R = (128, 128, 128, 128), 32
    print(f"case dense 128^4 R=32 gradient rows {prec}", flush=True)
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=0, dtype=np.float32)
    Tg = cpng.Tensor(dims, torch.from_numpy(p.T).cuda().reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    u0 = initial_guess(dims, R, seed=10000)
    A = ocp.split_u(u0, dims, R)
    _, g = cpng.cp_objective_grad(h, Tg, torch.from_numpy(u0).cuda(), R, prec)
    G = ocp.split_u(g.cpu().numpy(), dims, R)
    grams = [a.T @ a for a in A]
    rows = [0, 77, 127]
    for n in range(4):
        sl = np.take(p.T, rows, axis=n).astype(np.float64)
        An = [a if k != n else A[n][rows] for k, a in enumerate(A)]
        gb = np.ones((R, R))
        for k in range(4):
            if k != n:
                gb = gb * grams[k]
        ref = -ocp.mttkrp(sl, An, n) + A[n][rows] @ gb
        bound = (ocp.mttkrp(np.abs(sl), [np.abs(a) for a in An], n)
                 + np.abs(A[n][rows]) @ np.abs(gb))
        assert_close_to_bound(G[n][rows], ref, bound, TOL[prec], f"mode {n} {prec}")


def test_sparse_20000x3_R16_sampled_rows(h):
    import paper_1105_5331_amd as cpng
    dims, R = (20000, 20000, 20000), 16
    print("case sparse 20000^3 nnz~2e7 R=16 full size", flush=True)
    sp = sparse_random_cp(dims, 20_000_000, 16, seed=0, dtype=np.float32)
    Tg = cpng.Tensor(dims, torch.from_numpy(sp.values).cuda(),
                     coords=torch.from_numpy(sp.coords).cuda())
    cpng.cp_tensor_prepare(h, Tg)
    rng = np.random.default_rng(1)
    A = [rng.standard_normal((I, R)) for I in dims]
    u = torch.from_numpy(ocp.join_u(A)).cuda()
    vals = sp.values.astype(np.float64)
    for n in range(3):
        M = cpng.cp_mttkrp(h, Tg, u, R, n, "fp32").cpu().numpy()
        rows = np.array([0, 4321, 19999, int(sp.coords[n, 12345])])
        for i in rows:
            sel = sp.coords[n] == i
            ref = ocp.mttkrp_coo(dims, sp.coords[:, sel], vals[sel], A, n)[i]
            bound = ocp.mttkrp_coo(dims, sp.coords[:, sel], np.abs(vals[sel]),
                                   [np.abs(a) for a in A], n)[i]
            assert_close_to_bound(M[i][None], ref[None], bound[None], TOL["fp32"],
                                  f"mode {n} row {i}")
    cpng.cp_tensor_release(h, Tg)


@pytest.mark.parametrize("prec,tol", [("fp64", 1e-12), ("fp32in_fp64acc", 1e-12),
                                      ("fp32", 1e-5), ("bf16x3", 1e-4)])
def test_dense_200x3_R10_objective_grad(h, prec, tol):
    """|df| / (1/2 ||T||^2 + |f|) and ||dg|| / (||T|| + ||g||) against the
    oracle on the same tensor (float64 for "fp64", the float32 tensor widened
    otherwise).  At the random initial guess f is about 2e5 (1/2 ||T||^2), and
    the rounding of f and g scales with the terms they are formed from."""
    import paper_1105_5331_amd as cpng
    dims, R = (200, 200, 200), 10
    print(f"case dense 200^3 R=10 objective/gradient {prec}", flush=True)
    p = test_problem_1(dims, R, 0.9, 1, 1, seed=0, dtype=np.float64 if prec == "fp64" else np.float32)
    T64 = p.T.astype(np.float64)
    Tg = cpng.Tensor(dims, torch.from_numpy(p.T).cuda().reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    u0 = initial_guess(dims, R, seed=10000)
    A = ocp.split_u(u0, dims, R)
    f, g = cpng.cp_objective_grad(h, Tg, torch.from_numpy(u0).cuda(), R, prec)
    half = 0.5 * float(np.sum(T64 ** 2))
    fo = ocp.objective_direct(T64, A)
    go = ocp.join_u(ocp.gradient_from_mttkrps(A, [ocp.mttkrp(T64, A, n) for n in range(3)]))
    assert abs(f.item() - fo) / (half + abs(fo)) <= tol
    assert np.linalg.norm(g.cpu().numpy() - go) / (np.sqrt(2 * half) + np.linalg.norm(go)) <= tol
