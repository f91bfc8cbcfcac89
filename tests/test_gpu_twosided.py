"""One-pass evaluation: both group partials of the two-level evaluation from a
single read of T (the two-sided kernel), checked through cp_objective_grad
against the float64 oracle element by element (Section 2.3's f and g from
all N MTTKRPs at one point), in every precision class the kernel has.

Covered shapes: float32 tensor, order >= 4 with both mode groups of more than
one mode, the last mode of each group of length 64 or 128, R <= 32.  The
cases span one and several 32-row chunks per slab, both slab widths, outer
groups of one and of two modes (order 5), R = 1, R = 32 and ranks that leave
part of a 16-wide rank tile empty, outer counts that leave the last
workgroup with fewer outer indices than the others, and left outer counts
that 4 divides (four outer indices per workgroup) and that it does not (two)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cp as ocp
from workloads import initial_guess, test_problem_1

from helpers import TOL, assert_close_to_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_1105_5331_amd as cpng
    with cpng.Handle(0) as handle:
        yield handle


def _dev(x):
    return torch.from_numpy(np.ascontiguousarray(x)).cuda()


# (dims, R): split before mode 2 for the order-4 shapes, before mode 3 for the order-5 one
# (2, 64, 515, 64): two outer indices on the left, 515 on the right, more
# than the workgroups take one each, so the last workgroup gets fewer than
# the rest; left outer counts 8, 4, 12 and (order 5) 4 x 2 run four per
# workgroup, the others two
CASES = [((8, 64, 6, 128), 5), ((4, 128, 3, 64), 32), ((2, 3, 64, 4, 128), 7),
         ((6, 128, 5, 128), 17), ((2, 64, 3, 64), 1), ((10, 64, 9, 128), 16),
         ((2, 64, 515, 64), 9), ((12, 64, 5, 128), 32), ((4, 2, 64, 7, 64), 11)]
PRECS = ["bf16x3", "fp32", "fp32in_fp64acc", "fp64"]


def _kernel_ids(cpng, prec):
    if prec in ("bf16x3", "fp32"):
        return cpng.CP_KERNEL_DENSE_TWOSIDED, cpng.CP_KERNEL_DENSE_MTTKRP
    return cpng.CP_KERNEL_DENSE_TWOSIDED_F64, cpng.CP_KERNEL_DENSE_MTTKRP_F64


@pytest.mark.parametrize("dims,R", CASES)
@pytest.mark.parametrize("prec", PRECS)
def test_one_pass_objective_grad(h, dims, R, prec):
    """f and every element of g from one pass over T against the oracle: the
    gradient within tol x (|T|-weighted MTTKRP bound + |A| |Gammabar|), f
    within tol x (1/2 ||T||^2 + |f|); one two-sided launch and no
    single-partial launch."""
    import paper_1105_5331_amd as cpng
    print(f"case one-pass objective_grad dims={dims} R={R} prec={prec}", flush=True)
    N = len(dims)
    p = test_problem_1(dims, R, 0.6, 1, 1, seed=9, dtype=np.float32)
    T64 = p.T.astype(np.float64)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    A = [0.5 * a for a in ocp.split_u(initial_guess(dims, R, seed=77), dims, R)]
    two, single = _kernel_ids(cpng, prec)
    cpng.cp_profile_select(h, (1 << two) | (1 << single))
    cpng.cp_profile(h, True)
    f, g = cpng.cp_objective_grad(h, Tg, _dev(ocp.join_u(A)), R, prec)
    torch.cuda.synchronize()
    n_two, _ = cpng.cp_profile_read(h, two)
    n_single, _ = cpng.cp_profile_read(h, single)
    cpng.cp_profile(h, False)
    cpng.cp_profile_select(h, 0xFF)
    assert (n_two, n_single) == (1, 0)
    Ms = [ocp.mttkrp(T64, A, n) for n in range(N)]
    G = ocp.split_u(g.cpu().numpy(), dims, R)
    Gref = ocp.gradient_from_mttkrps(A, Ms)
    absA = [np.abs(a) for a in A]
    for n in range(N):
        gb = np.ones((R, R))
        for k in range(N):
            if k != n:
                gb = gb * (absA[k].T @ absA[k])
        bound = ocp.mttkrp(np.abs(T64), absA, n) + absA[n] @ gb
        assert_close_to_bound(G[n], Gref[n], bound, TOL[prec], f"mode {n} {prec}")
    half = 0.5 * float(np.sum(T64 ** 2))
    fo = ocp.objective_direct(T64, A)
    assert abs(f.item() - fo) <= TOL[prec] * (half + abs(fo))


def test_uncovered_shapes_take_two_passes(h):
    """Shapes the two-sided kernel does not cover (a group's last mode of
    another length, R above 32, an odd left outer count) run the two
    single-partial passes."""
    import paper_1105_5331_amd as cpng
    for dims, R in [((4, 96, 3, 64), 5), ((4, 64, 3, 128), 33), ((4, 64, 3, 40), 3),
                    ((3, 64, 4, 64), 5)]:
        print(f"case two-pass fallback dims={dims} R={R}", flush=True)
        p = test_problem_1(dims, min(R, 8), 0.5, 1, 1, seed=2, dtype=np.float32)
        Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
        cpng.cp_tensor_prepare(h, Tg)
        u = _dev(initial_guess(dims, R, seed=5))
        cpng.cp_profile_select(h, (1 << cpng.CP_KERNEL_DENSE_TWOSIDED) |
                               (1 << cpng.CP_KERNEL_DENSE_MTTKRP))
        cpng.cp_profile(h, True)
        cpng.cp_objective_grad(h, Tg, u, R, "bf16x3")
        torch.cuda.synchronize()
        n_two, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_TWOSIDED)
        n_single, _ = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_MTTKRP)
        cpng.cp_profile(h, False)
        cpng.cp_profile_select(h, 0xFF)
        assert n_two == 0 and n_single == 2, (dims, R, n_two, n_single)


@pytest.mark.parametrize("prec", ["bf16x3", "fp32in_fp64acc"])
def test_one_pass_is_reproducible(h, prec):
    """Two evaluations at the same point give the same bits (fixed-order
    split-K slots, no atomics)."""
    import paper_1105_5331_amd as cpng
    dims, R = (10, 64, 9, 128), 16
    print(f"case one-pass bitwise repeat {prec}", flush=True)
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=4, dtype=np.float32)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    u = _dev(initial_guess(dims, R, seed=8))
    f1, g1 = cpng.cp_objective_grad(h, Tg, u, R, prec)
    f2, g2 = cpng.cp_objective_grad(h, Tg, u, R, prec)
    assert f1.item() == f2.item()
    assert torch.equal(g1, g2)


# (64, 128, 40, 128), R = 32: the iterate is long enough for the multi-kernel
# normalisation (the reused left partial is rescaled from its plan in global
# memory); (8, 64, 6, 128): the one-workgroup normalisation
@pytest.mark.parametrize("dims,R", [((8, 64, 6, 128), 6), ((64, 128, 40, 128), 32)])
@pytest.mark.parametrize("prec", ["fp32in_fp64acc", "bf16x3"])
def test_trajectory_one_pass_vs_two_passes(h, prec, dims, R):
    """N-GMRES with the one-pass evaluation (mttkrp_tree = 1) against the same
    run with a pass per partial (mttkrp_tree = 2): the per-iterate objective
    agrees to the evaluation's rounding over the first iterations, and each
    evaluation makes one pass instead of two; the ALS sweep makes one where
    it takes its left partial from the last evaluation (that evaluation was
    at the sweep's starting point: the first step, after a restart or a line
    search converged on its last trial), two otherwise."""
    import paper_1105_5331_amd as cpng
    print(f"case one-pass trajectory {prec} dims={dims} R={R}", flush=True)
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=1, dtype=np.float32)
    Tg = cpng.Tensor(dims, _dev(p.T).reshape(-1))
    cpng.cp_tensor_prepare(h, Tg)
    u0 = initial_guess(dims, R, seed=10001)
    runs = {}
    for tree in (1, 2):
        st = cpng.NGMRESState(h, Tg, R, _dev(u0), precision=prec, final_precision=prec,
                              mttkrp_tree=tree)
        runs[tree] = [st.step() for _ in range(6)]
        st.close()
    half = 0.5 * Tg.norm_sq
    ftol = 1e-11 if prec == "fp32in_fp64acc" else 1e-4
    for k, (a, b) in enumerate(zip(runs[1], runs[2])):
        assert abs(a["f"] - b["f"]) <= ftol * half, (k, a["f"], b["f"])
    # a sweep of one pass follows a step that ended on its last evaluated point
    # (a restart, or the accepted step is the last trial); the first step's
    # sweep starts from the created state's evaluation
    sweeps = [a["t_passes"] - 1 - a["nfev"] for a in runs[1]]
    assert all(sw in (1, 2) for sw in sweeps), sweeps
    assert sweeps[0] == 1 and sum(sw == 1 for sw in sweeps) >= 2, sweeps
    for k, a in enumerate(runs[1][1:], start=1):
        if runs[1][k - 1]["restart"] or runs[1][k - 1]["ls_status"] == "converged":
            assert sweeps[k] == 1, (k, sweeps)
    for k, b in enumerate(runs[2]):
        assert b["t_passes"] == 2 * (2 + b["nfev"]), (k, b)
