"""cp_mttkrp_noalloc: the MTTKRP whose workspace is the library's static
per-device scratch array instead of allocated memory.

Checked through the C ABI against cp_mttkrp (the same kernels on the handle's
grown workspace: bitwise equal outputs) and against the float64 oracle, on two
calls in a row whose second input is smaller than the first; sparse tensors
too; a call whose workspace would exceed the array is rejected with CP_ENOMEM
before anything is launched; and the calls leave the device's free memory
unchanged where cp_mttkrp on a fresh handle grows its workspace.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from oracle import cp as ocp
from workloads import initial_guess, random_coo, test_problem_1, test_problem_1_torch

from helpers import TOL, abs_mttkrp, abs_mttkrp_coo, assert_close_to_bound

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def h():
    import paper_1105_5331_amd as cpng
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a GPU")
    with cpng.Handle(0) as handle:
        yield handle


def _dense(dims, R, seed, dtype):
    p = test_problem_1(dims, R, 0.5, 1, 1, seed=seed, dtype=dtype)
    u0 = initial_guess(dims, R, seed=seed + 10000)
    return p.T, u0


# (larger, smaller) pairs: each pair runs in this order on the no-alloc entry
PAIRS = [
    (((96, 80, 72), 16), ((20, 20, 20), 3)),
    (((40, 36, 32, 24), 33), ((7, 9, 5, 11), 5)),
    (((130, 7, 24, 16), 10), ((33, 17, 45), 1)),
]


@pytest.mark.parametrize("prec", ["fp64", "fp32", "bf16x3", "fp32in_fp64acc"])
@pytest.mark.parametrize("pair", PAIRS, ids=lambda p: "x".join(map(str, p[0][0])))
def test_noalloc_matches_cp_mttkrp_two_calls(h, pair, prec):
    import paper_1105_5331_amd as cpng
    dtype = np.float64 if prec == "fp64" else np.float32
    for (dims, R) in pair:   # larger first, then smaller
        print(f"case noalloc dense dims={dims} R={R} prec={prec}", flush=True)
        T, u0 = _dense(dims, R, 3, dtype)
        Tg = cpng.Tensor(dims, torch.from_numpy(T).cuda().reshape(-1))
        u = torch.from_numpy(u0).cuda()
        A = ocp.split_u(u0, dims, R)
        T64 = T.astype(np.float64)
        for n in range(len(dims)):
            M0 = cpng.cp_mttkrp_noalloc(h, Tg, u, R, n, prec)
            M1 = cpng.cp_mttkrp(h, Tg, u, R, n, prec)
            torch.cuda.synchronize()
            M0, M1 = M0.cpu().numpy(), M1.cpu().numpy()
            assert np.array_equal(M0.view(np.uint64), M1.view(np.uint64)), f"mode {n}: not bitwise"
            ref = ocp.mttkrp(T64, A, n)
            assert_close_to_bound(M0, ref, abs_mttkrp(T64, A, n), TOL[prec], f"mode {n}")


@pytest.mark.parametrize("prec", ["fp32", "fp64"])
def test_noalloc_sparse_two_calls(h, prec):
    import paper_1105_5331_amd as cpng
    for dims, nnz, R, seed in [((300, 40, 50), 9000, 16, 2), ((7, 8, 9), 100, 3, 1)]:
        print(f"case noalloc sparse dims={dims} nnz={nnz} R={R} prec={prec}", flush=True)
        sp = random_coo(dims, nnz, seed=seed, dtype=np.float32 if prec == "fp32" else np.float64)
        vals = torch.from_numpy(sp.values).cuda()
        coords = torch.from_numpy(sp.coords.astype(np.int32)).cuda()
        Tg = cpng.Tensor(dims, vals, coords)
        cpng.cp_tensor_prepare(h, Tg)
        rng = np.random.default_rng(seed)
        A = [rng.standard_normal((I, R)) for I in dims]
        u = torch.from_numpy(ocp.join_u(A)).cuda()
        v64 = sp.values.astype(np.float64)
        for n in range(len(dims)):
            M0 = cpng.cp_mttkrp_noalloc(h, Tg, u, R, n, prec)
            M1 = cpng.cp_mttkrp(h, Tg, u, R, n, prec)
            torch.cuda.synchronize()
            M0, M1 = M0.cpu().numpy(), M1.cpu().numpy()
            assert np.array_equal(M0.view(np.uint64), M1.view(np.uint64)), f"mode {n}: not bitwise"
            ref = ocp.mttkrp_coo(dims, sp.coords, v64, A, n)
            bound = abs_mttkrp_coo(dims, sp.coords, v64, A, n)
            assert_close_to_bound(M0, ref, bound, TOL[prec], f"mode {n}")
        cpng.cp_tensor_release(h, Tg)


def test_noalloc_full_size_128x4_R32(h):
    """The benchmark's dense shape (1 GB float32 tensor, R = 32): its largest
    workspace (BF16X3, about 19 MB) fits the array; bitwise equal to
    cp_mttkrp in every mode, then a smaller call."""
    import paper_1105_5331_amd as cpng
    dims, R = (128, 128, 128, 128), 32
    print("case noalloc dense 128^4 R=32", flush=True)
    Tg = cpng.Tensor(dims, test_problem_1_torch(dims, R, 0.5, seed=0))
    u = torch.from_numpy(initial_guess(dims, R, seed=10000)).cuda()
    for prec in ("bf16x3", "fp32"):
        for n in range(4):
            M0 = cpng.cp_mttkrp_noalloc(h, Tg, u, R, n, prec)
            M1 = cpng.cp_mttkrp(h, Tg, u, R, n, prec)
            torch.cuda.synchronize()
            assert torch.equal(M0.view(torch.int64), M1.view(torch.int64)), f"{prec} mode {n}"
    del Tg
    dims, R = (24, 8, 16), 4
    T, u0 = _dense(dims, R, 1, np.float32)
    Tg = cpng.Tensor(dims, torch.from_numpy(T).cuda().reshape(-1))
    u = torch.from_numpy(u0).cuda()
    A = ocp.split_u(u0, dims, R)
    for n in range(3):
        M0 = cpng.cp_mttkrp_noalloc(h, Tg, u, R, n, "bf16x3").cpu().numpy()
        ref = ocp.mttkrp(T.astype(np.float64), A, n)
        assert_close_to_bound(M0, ref, abs_mttkrp(T.astype(np.float64), A, n), TOL["bf16x3"],
                              f"mode {n}")


def test_noalloc_rejects_workspace_beyond_the_array(h):
    """FP32 stages the factors as float32 first: with L = 32 * (2^20 + 8)
    that is 134 MB, beyond the 64 MiB array -> CP_ENOMEM before any launch;
    the next call still works."""
    import paper_1105_5331_amd as cpng
    from paper_1105_5331_amd._native import CP_ENOMEM
    dims, R = (4, 4, 1 << 20), 32
    print("case noalloc oversize", flush=True)
    T = torch.ones(dims, dtype=torch.float32, device="cuda").reshape(-1)
    Tg = cpng.Tensor(dims, T)
    u = torch.full((sum(dims) * R,), 0.5, dtype=torch.float64, device="cuda")
    with pytest.raises(cpng.CpError) as e:
        cpng.cp_mttkrp_noalloc(h, Tg, u, R, 0, "fp32")
    assert e.value.code == CP_ENOMEM
    assert "static scratch" in str(e.value)
    del Tg, T, u
    dims, R = (20, 20, 20), 3
    Tn, u0 = _dense(dims, R, 2, np.float32)
    Tg = cpng.Tensor(dims, torch.from_numpy(Tn).cuda().reshape(-1))
    u = torch.from_numpy(u0).cuda()
    A = ocp.split_u(u0, dims, R)
    M0 = cpng.cp_mttkrp_noalloc(h, Tg, u, R, 1, "fp32").cpu().numpy()
    ref = ocp.mttkrp(Tn.astype(np.float64), A, 1)
    assert_close_to_bound(M0, ref, abs_mttkrp(Tn.astype(np.float64), A, 1), TOL["fp32"], "after")


def test_noalloc_leaves_free_memory_unchanged():
    """On a fresh handle (no workspace grown yet), no-alloc calls leave the
    device's free memory where it was; cp_mttkrp on another fresh handle
    grows the handle's workspace by megabytes (the check can see it)."""
    import paper_1105_5331_amd as cpng
    dims, R = (128, 128, 64, 64), 32
    print("case noalloc free memory", flush=True)
    Tg = cpng.Tensor(dims, test_problem_1_torch(dims, R, 0.5, seed=4))
    u = torch.from_numpy(initial_guess(dims, R, seed=10004)).cuda()
    outs = [torch.empty((dims[n], R), dtype=torch.float64, device="cuda") for n in range(4)]
    with cpng.Handle(0) as hw:   # load every kernel once (code objects, launch resources)
        for n in range(4):
            cpng.cp_mttkrp_noalloc(hw, Tg, u, R, n, "bf16x3", M_out=outs[n])
            cpng.cp_mttkrp(hw, Tg, u, R, n, "bf16x3", M_out=outs[n])
        torch.cuda.synchronize()
    with cpng.Handle(0) as h1:
        torch.cuda.synchronize()
        free0 = torch.cuda.mem_get_info()[0]
        for n in range(4):
            cpng.cp_mttkrp_noalloc(h1, Tg, u, R, n, "bf16x3", M_out=outs[n])
        torch.cuda.synchronize()
        free1 = torch.cuda.mem_get_info()[0]
    assert free1 == free0, (free0, free1)
    with cpng.Handle(0) as h2:
        torch.cuda.synchronize()
        free2 = torch.cuda.mem_get_info()[0]
        for n in range(4):
            cpng.cp_mttkrp(h2, Tg, u, R, n, "bf16x3", M_out=outs[n])
        torch.cuda.synchronize()
        free3 = torch.cuda.mem_get_info()[0]
    assert free2 - free3 >= 4 << 20, (free2, free3)
