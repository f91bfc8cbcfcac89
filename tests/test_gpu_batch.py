"""The batched N-GMRES path for small dense requests (cp_batch_decompose),
through the C ABI: every request of a batch follows the FP64 oracle's
trajectory from the same initial guess (float32 tensors, widened exactly on
both sides), a request's result is bitwise the same alone and in a batch, and
requests outside the path's limits are rejected.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cp as ocp
from oracle.ngmres import CPProblem, ngmres
from workloads import initial_guess, test_problem_1

from helpers import compare_trajectory as _compare

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_1105_5331_amd as cpng
    with cpng.Handle(0) as handle:
        yield handle


# (dims, R, congruence, seed): orders 3 and 4, ragged sizes, ranks 1..32
CASES = [((20, 20, 20), 3, 0.5, 0), ((12, 17, 9), 5, 0.9, 1), ((9, 11, 8, 10), 3, 0.5, 2),
         ((30, 7, 25), 1, 0.0, 3), ((16, 16, 16), 12, 0.5, 4), ((6, 7, 5, 8), 2, 0.3, 5),
         ((40, 24, 16), 32, 0.2, 6)]


def _problems(cases):
    out = []
    for dims, R, c, seed in cases:
        p = test_problem_1(dims, R, c, 1, 1, seed=seed, dtype=np.float32)
        out.append((dims, R, p.T, initial_guess(dims, R, seed=seed + 10000)))
    return out


def _run(h, probs, max_iter, trace_cap=0, **opts):
    import paper_1105_5331_amd as cpng
    Ts, us = [], []
    for dims, R, T, u0 in probs:
        Tg = cpng.Tensor(dims, torch.from_numpy(T).cuda().reshape(-1))
        cpng.cp_tensor_prepare(h, Tg)
        Ts.append(Tg)
        us.append(torch.from_numpy(u0).cuda())
    res = cpng.cp_batch_decompose(h, Ts, [p[1] for p in probs], 1e-8, us, trace_cap=trace_cap,
                                  max_iter=max_iter, **opts)
    torch.cuda.synchronize()
    return res, [u.cpu().numpy() for u in us]


def test_batch_trajectories_follow_the_oracle(h):
    """Iterate by iterate (f, rho, beta) until the first discrete divergence,
    over at most the first 100 iterates: the congruence-0.9 case converges in
    166 iterations, and past about 100 the oracle against itself with u0
    perturbed by 1e-15 moves rho by up to 60% (within the first 100: f by
    9e-13 of 1/2 ||T||^2, rho by 1.4e-7 relative); every other case converges
    well within 100."""
    print("case batch trajectories", flush=True)
    probs = _problems(CASES)
    res, _ = _run(h, probs, max_iter=200, trace_cap=260)
    for (dims, R, T, u0), r in zip(probs, res):
        T64 = T.astype(np.float64)
        ref = ngmres(CPProblem(ocp.DenseTensor(T64), R), u0, tol=1e-8, max_iter=200)
        half = 0.5 * float(np.sum(T64 ** 2))
        n = _compare(r["trace"][:100], ref.trace[:100], half, f"batch {dims} R={R}")
        # a run of a few iterations ends near the stopping tolerance, where
        # a restart can be decided by rounding: at least all but the last two
        assert n >= min(len(ref.trace) - 2, 5), (dims, R, n)
        assert r["status"] in (0, 1)
        if ref.converged:
            assert r["converged"], (dims, R, r["rho"])


def test_batch_result_is_the_same_alone_and_in_a_batch(h):
    print("case batch isolation", flush=True)
    probs = _problems(CASES)
    together, u_all = _run(h, probs, max_iter=120, trace_cap=130)
    for k, p in enumerate(probs):
        alone, u_one = _run(h, [p], max_iter=120, trace_cap=130)
        assert np.array_equal(u_one[0].view(np.uint64), u_all[k].view(np.uint64)), p[0]
        a, b = alone[0], together[k]
        assert (a["iters"], a["f"], a["rho"], a["n_fg"]) == (b["iters"], b["f"], b["rho"], b["n_fg"])
        assert [t["f"] for t in a["trace"]] == [t["f"] for t in b["trace"]]


def test_batch_line_search_fallback_follows_the_oracle(h):
    """Every search capped at two trials with a curvature tolerance no trial
    meets: each ends without a Wolfe point and takes the better trial (kept
    gradient) or beta = 0, on both sides; compared while rho > 1e-4."""
    print("case batch line-search fallback", flush=True)
    probs = _problems([((20, 20, 20), 3, 0.5, 3), ((10, 12, 9, 8), 4, 0.5, 7)])
    res, _ = _run(h, probs, max_iter=40, trace_cap=60, ls_maxfev=2, ls_gtol=1e-12)
    for (dims, R, T, u0), r in zip(probs, res):
        T64 = T.astype(np.float64)
        ref = ngmres(CPProblem(ocp.DenseTensor(T64), R), u0, tol=1e-8, max_iter=40,
                     ls=dict(maxfev=2, gtol=1e-12))
        window = [t for t in ref.trace if t.rho > 1e-4]
        assert window == ref.trace[:len(window)] and len(window) >= 5
        half = 0.5 * float(np.sum(T64 ** 2))
        n = _compare(r["trace"], window, half, f"batch fallback {dims}")
        assert n == len(window)
        assert r["n_ls_fallback"] >= 3


def test_batch_rejects_requests_outside_its_limits(h):
    import paper_1105_5331_amd as cpng
    p = test_problem_1((6, 7, 5), 40, 0.5, 1, 1, seed=1, dtype=np.float32)
    Tg = cpng.Tensor((6, 7, 5), torch.from_numpy(p.T).cuda().reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    u = torch.rand(18 * 40, dtype=torch.float64, device="cuda")
    with pytest.raises(cpng.CpError):   # R = 40 > 32
        cpng.cp_batch_decompose(h, [Tg], [40], 1e-8, [u])
    T2 = torch.rand(64, dtype=torch.float32, device="cuda")
    Tg2 = cpng.Tensor((8, 8), T2)
    cpng.cp_tensor_prepare(h, Tg2)
    u2 = torch.rand(16 * 2, dtype=torch.float64, device="cuda")
    with pytest.raises(cpng.CpError):   # order 2
        cpng.cp_batch_decompose(h, [Tg2], [2], 1e-8, [u2])
