"""GPU tests of the continuous-batching server (cp_server_* in the C ABI):
every request finishes, admission respects the HBM budget, and each result
is bitwise the same when the request runs alone and when it runs in a mix."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from workloads import initial_guess, serving_stream, test_problem_1, test_problem_1_torch

pytestmark = pytest.mark.gpu


def _requests(n, seed=3):
    reqs = serving_stream(n, rate_per_s=100.0, seed=seed, size_range=(16, 48))
    out = []
    for r in reqs:
        T = test_problem_1_torch(r.dims, r.R, r.c, 1, 1, seed=r.seed)
        u0 = torch.from_numpy(initial_guess(r.dims, r.R, seed=r.seed + 10000)).cuda()
        out.append((r, T, u0))
    return out


def _run(reqs, slots, **opts):
    import paper_1105_5331_amd as cpng
    results = {}
    with cpng.Server(0, slots=slots, max_iter=300, **opts) as srv:
        us = {}
        for r, T, u0 in reqs:
            u = u0.clone()
            us[r.rid] = u
            srv.submit(cpng.Tensor(r.dims, T), r.R, 1e-8, u, tag=r.rid)
        got = []
        while len(got) < len(reqs):
            got += srv.poll(wait_for=len(reqs) - len(got))
        for g in got:
            results[g["tag"]] = (g, us[g["tag"]].cpu().numpy())
    return results


def test_isolation_alone_vs_mix_bitwise():
    reqs = _requests(12)
    mix = _run(reqs, slots=4)
    for i in range(0, 12, 3):            # a subset, each run alone
        alone = _run([reqs[i]], slots=1)
        a_res, a_u = alone[reqs[i][0].rid]
        m_res, m_u = mix[reqs[i][0].rid]
        assert a_res["status"] == m_res["status"]
        assert a_res["iters"] == m_res["iters"]
        assert np.array_equal(a_u, m_u), f"request {i} differs alone vs in the mix"
        assert a_res["rho"] == m_res["rho"]


def test_isolation_50_requests_one_at_a_time_vs_mix():
    """50 requests of the serving mix: run one at a time (a single slot, so no
    other request is ever on the device with it) and as a 4-slot mix, every
    result is the same bits."""
    print("case serving isolation, 50 requests", flush=True)
    reqs = _requests(50, seed=11)
    alone = _run(reqs, slots=1)
    mix = _run(reqs, slots=4)
    assert len(alone) == len(mix) == 50
    for r, _, _ in reqs:
        a_res, a_u = alone[r.rid]
        m_res, m_u = mix[r.rid]
        assert a_res["status"] == m_res["status"] and a_res["iters"] == m_res["iters"], r.rid
        assert a_res["rho"] == m_res["rho"], r.rid
        assert np.array_equal(a_u, m_u), f"request {r.rid} differs one at a time vs in the mix"


def test_isolation_with_the_batched_path_50_requests():
    """50 requests of the serving mix with the batched path on for tensors of
    at most 2^17 entries: run with one slot and a batch of one place (every
    batched request alone in its batch) and as a 4-slot mix with a full batch,
    every result is the same bits; both paths are used."""
    print("case serving isolation with the batched path", flush=True)
    reqs = _requests(50, seed=13)
    serial = _run(reqs, slots=1, batch_elems=1 << 17, batch_capacity=1)
    mix = _run(reqs, slots=4, batch_elems=1 << 17)
    assert len(serial) == len(mix) == 50
    n_batched = sum(1 for g, _ in mix.values() if g["slot"] == -1)
    assert 0 < n_batched < 50
    for r, _, _ in reqs:
        a_res, a_u = serial[r.rid]
        m_res, m_u = mix[r.rid]
        assert a_res["slot"] == -1 if m_res["slot"] == -1 else a_res["slot"] >= 0
        assert a_res["status"] == m_res["status"] and a_res["iters"] == m_res["iters"], r.rid
        assert a_res["rho"] == m_res["rho"], r.rid
        assert np.array_equal(a_u, m_u), f"request {r.rid} differs alone vs in the mix"
        if m_res["slot"] == -1:
            assert m_res["status"] in (0, 1) and np.all(np.isfinite(m_u))


def test_every_request_terminates_and_mixed_precision_certifies():
    reqs = _requests(10, seed=5)
    res = _run(reqs, slots=3, precision="bf16x3", final_precision="fp32in_fp64acc",
               switch_rho=1e-4)
    assert len(res) == 10
    for tag, (r, u) in res.items():
        assert r["status"] in (0, 1)          # CP_OK or CP_MAXITER
        assert np.all(np.isfinite(u))
        if r["converged"]:
            assert r["rho"] <= 1e-8


def test_admission_respects_budget():
    import paper_1105_5331_amd as cpng
    reqs = _requests(6, seed=7)
    # a budget that admits only about one request at a time
    with cpng.Server(0, slots=4, hbm_budget=200 << 20, max_iter=50) as srv:
        us = {}
        for r, T, u0 in reqs:
            u = u0.clone()
            us[r.rid] = u
            srv.submit(cpng.Tensor(r.dims, T), r.R, 1e-8, u, tag=r.rid)
        peak = 0
        got = []
        while len(got) < len(reqs):
            st = srv.stats()
            assert st["in_use"] <= st["budget"]
            peak = max(peak, st["active"])
            got += srv.poll(wait_for=1)
        assert all(g["status"] in (0, 1) for g in got)


def test_request_larger_than_budget_is_rejected():
    import paper_1105_5331_amd as cpng
    r, T, u0 = _requests(1, seed=9)[0]
    with cpng.Server(0, slots=1, hbm_budget=1 << 20) as srv:
        srv.submit(cpng.Tensor(r.dims, T), r.R, 1e-8, u0.clone(), tag=0)
        got = srv.poll(wait_for=1)
        assert got[0]["status"] == -2
