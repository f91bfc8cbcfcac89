#!/usr/bin/env python3
"""Benchmark of the N-GMRES/ALS hot path on one MI355X.

Workload (default): dense 4-way 128x128x128x128 float32 tensor (268,435,456
entries, 1.07 GB), rank R = 32, column congruence 0.5, noise l1 = l2 = 1
(Test Problem I generalised to four modes), seed 0; initial guess U[0,1)
seed 10000.  One "step" is one N-GMRES iteration through the C ABI
(ngmres_step): Step I (ALS sweep: N single-mode MTTKRPs with their Gram and
Cholesky solves), Step II (gradient at u_bar: N MTTKRPs, the window's normal
equations), Step III (line search: N MTTKRPs per trial).

value  = tensor bytes streamed by all MTTKRPs of the timed steps / wall time
         (GB/s, whole-job throughput, inputs resident in HBM).
roofline = the dense MTTKRP kernel alone: algorithmic bytes per launch
         (4 * #T + factor rows read + output) over its mean duration, timed
         with HIP events on the stream it runs on, against 8 TB/s.
cpu_baseline = the FP64 oracle's MTTKRP (all four modes) on a slab of the
         same tensor, on the host cores.
extra.time_to_grad = dense 200^3 float32, R = 10, congruence 0.9: wall time of
         cp_decompose to ||g||/||T|| <= 1e-8 with the plain FP64 GPU method
         (float64 tensor) versus the mixed method (float32 tensor, reduced-
         precision bulk, float64 accumulation for the tail), equal final h.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

PEAK_HBM_GBS = 8000.0


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(T, A, budget_s=12.0):
    """Oracle MTTKRP over a slab T[:s] (all modes), timed on the host cores."""
    from oracle import cp as ocp
    threads = os.cpu_count() or 1
    try:
        from threadpoolctl import threadpool_info
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [threads])
    except Exception:
        pass
    s = 2
    while True:
        slab = np.ascontiguousarray(T[:s], dtype=np.float64)
        Af = [A[0][:s]] + A[1:]
        t0 = time.perf_counter()
        for n in range(T.ndim):
            ocp.mttkrp(slab, Af, n)
        dt = time.perf_counter() - t0
        if dt * 2 > budget_s or s * 2 > T.shape[0]:
            break
        s *= 2
    bytes_ = 4.0 * slab.size * T.ndim       # float32 tensor bytes per pass, one pass per mode
    return {"value": bytes_ / dt / 1e9, "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"oracle MTTKRP of every mode on slab T[:{s}] ({slab.size} entries, "
                      f"float64 arithmetic) of the same tensor, {dt:.2f} s"}


def time_to_grad(h, cpng, torch, seed=0):
    from workloads import initial_guess, test_problem_1
    dims, R, tol = (200, 200, 200), 10, 1e-8
    p = test_problem_1(dims, R, 0.9, 1, 1, seed=seed, dtype=np.float32)
    T32 = torch.from_numpy(p.T).cuda().reshape(-1)
    T64 = T32.double()
    u0 = initial_guess(dims, R, seed=seed + 10000)
    out = {}
    for name, Tv, kw in [
        ("fp64", T64, dict(precision="fp64")),
        ("mixed_fp32", T32, dict(precision="fp32", final_precision="fp32in_fp64acc", switch_rho=1e-6)),
        ("mixed_bf16x3", T32, dict(precision="bf16x3", final_precision="fp32in_fp64acc", switch_rho=1e-6)),
    ]:
        Tg = cpng.Tensor(dims, Tv)
        cpng.cp_tensor_prepare(h, Tg)
        u = torch.from_numpy(u0).cuda()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = cpng.cp_decompose(h, Tg, R, tol, u, max_iter=3000, **kw)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        hval = float(np.sqrt(max(0.0, 2 * r["f"]) / Tg.norm_sq))
        out[name] = {"seconds": round(dt, 4), "iters": r["iters"], "rho": r["rho"], "h": hval,
                     "converged": r["converged"], "n_fg": r["n_fg"], "switch_iter": r["switch_iter"]}
        log(f"time_to_grad {name}: {dt:.3f} s, {r['iters']} it, rho {r['rho']:.2e}, h {hval:.12f}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--precision", default="bf16x3", choices=["bf16x3", "fp32", "fp64"])
    ap.add_argument("--rank", type=int, default=32)
    ap.add_argument("--size", type=int, default=128)
    ap.add_argument("--skip-cpu", action="store_true")
    ap.add_argument("--skip-extra", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only; --gpus {args.gpus} is not supported "
              "(the multi-GPU sharding is a design, not part of this build)", file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1105_5331_amd as cpng
    from workloads import initial_guess, test_problem_1

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    s, R, N = args.size, args.rank, 4
    dims = (s,) * N
    log(f"generating dense {dims} float32 Test Problem I, R={R}")
    t0 = time.perf_counter()
    prob = test_problem_1(dims, R, 0.5, 1, 1, seed=0, dtype=np.float32)
    log(f"generated in {time.perf_counter() - t0:.1f} s")
    nT = prob.T.size
    T = torch.from_numpy(prob.T).cuda().reshape(-1)
    if args.precision == "fp64":
        T = T.double()
    u0 = initial_guess(dims, R, seed=10000)

    h = cpng.Handle(0)
    Tg = cpng.Tensor(dims, T)
    cpng.cp_tensor_prepare(h, Tg)
    st = cpng.NGMRESState(h, Tg, R, torch.from_numpy(u0).cuda(), precision=args.precision)
    for _ in range(args.warmup):
        st.step()
    torch.cuda.synchronize()
    log(f"warmup done ({args.warmup} steps)")
    cpng.cp_profile(h, True)
    torch.cuda.synchronize()
    passes = 0
    t0 = time.perf_counter()
    infos = []
    for k in range(args.steps):
        info = st.step()
        infos.append(info)
        passes += N * (2 + info["nfev"])
        log(f"step {k}: f {info['f']:.6e} rho {info['rho']:.3e} nfev {info['nfev']} "
            f"restart {info['restart']}")
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    launches, kms = cpng.cp_profile_read(h, cpng.CP_KERNEL_DENSE_MTTKRP)
    cpng.cp_profile(h, False)
    elem = 8 if args.precision == "fp64" else 4
    value = passes * nT * elem / dt / 1e9
    avg_ms = kms / max(1, launches)
    # algorithmic bytes of one single-mode MTTKRP launch: the tensor once, the
    # (N-1) factor copies it reads, the I_n x R output (float64)
    fac_bytes = (N - 1) * s * R * (8 if args.precision == "fp64" else 4)
    traffic = nT * elem + fac_bytes + s * R * 8
    achieved = traffic / (avg_ms * 1e-3) / 1e9
    res = {
        "metric": "MTTKRP HBM GB/s (% peak); time-to-grad-1e-8 vs FP64 GPU; serving p50/p99",
        "value": round(value, 2), "unit": "GB/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": round(dt / args.steps * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": {"bf16x3": "bf16x3", "fp32": "f32", "fp64": "f64"}[args.precision],
        "data": "synthetic",
        "config": {"workload": f"dense {s}^4 float32 Test Problem I, R={R}, congruence 0.5, "
                               f"noise 1%+1%, one N-GMRES iteration per step",
                   "dims": list(dims), "rank": R, "precision": args.precision,
                   "mttkrp_passes": passes},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": PEAK_HBM_GBS,
                     "unit": "GB/s", "frac": round(achieved / PEAK_HBM_GBS, 4), "traffic": None,
                     "kernel": "dense MTTKRP", "launches": launches,
                     "avg_us": round(avg_ms * 1e3, 2), "bytes_per_launch": traffic},
    }
    st.close()
    if not args.skip_extra:
        log("time-to-grad study (200^3, R=10, c=0.9)")
        res["extra"] = {"time_to_grad_200cubed_R10": time_to_grad(h, cpng, torch)}
    if not args.skip_cpu:
        log("cpu baseline (oracle)")
        A = [np.ascontiguousarray(x) for x in
             [u0[sum(dims[:k]) * R:sum(dims[:k + 1]) * R].reshape(dims[k], R) for k in range(N)]]
        res["cpu_baseline"] = cpu_baseline(prob.T, A)
    h.close()
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
