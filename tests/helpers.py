"""Shared helpers of the GPU parity tests (tolerances and conversions)."""
import numpy as np

from oracle import cp as ocp

# Element-wise MTTKRP tolerances, relative to the MTTKRP of |T| with |A|
# (the sum of absolute values of the terms of each output):
#   FP64 / FP32-in-FP64-acc: float64 products and sums, a few hundred
#     sequential additions per output at most -> well below 1e-12;
#   FP32: factor copies, products and per-workgroup sums rounded to float32
#     (unit roundoff 6e-8, a few hundred additions) -> 1e-5 (the per-iterate
#     float32 tolerance of the method's precision study);
#   BF16X3: split operands lose at most 3 * 2^-16 relative per product, plus
#     float32 accumulation -> 1e-4 element-wise, and 1e-3 on ||dM|| / ||M||.
TOL = {"fp64": 1e-12, "fp32in_fp64acc": 1e-12, "fp32": 1e-5, "bf16x3": 1e-4}


def abs_mttkrp(T, factors, n):
    return ocp.mttkrp(np.abs(T), [np.abs(a) for a in factors], n)


def abs_mttkrp_coo(dims, coords, values, factors, n):
    return ocp.mttkrp_coo(dims, coords, np.abs(values), [np.abs(a) for a in factors], n)


def assert_close_to_bound(got, ref, bound, tol, what=""):
    got = np.asarray(got)
    err = np.abs(got - ref)
    lim = tol * bound + 1e-300
    bad = err > lim
    if bad.any():
        i = np.unravel_index(np.argmax(err / lim), err.shape)
        raise AssertionError(f"{what}: {bad.sum()} elements over tolerance; worst at {i}: "
                             f"got {got[i]!r} ref {ref[i]!r} bound {bound[i]!r} tol {tol}")


# Per-iterate tolerances on a shared N-GMRES trajectory (float64 on both
# sides; the rationale -- the oracle's own sensitivity to rounding-level
# changes, amplified by the regularised normal equations -- is in the
# docstring of test_gpu_decompose.py):
F_TOL = 1e-10     # |f_gpu - f_oracle| / (1/2 ||T||^2)
RHO_REL = 1e-2    # |rho_gpu - rho_oracle| / rho_oracle ...
RHO_ABS = 1e-9    # ... + this absolute floor
BETA_REL = 1e-2   # |beta_gpu - beta_oracle| / max(1, |beta_oracle|)


def compare_trajectory(trace, ref_trace, half, what, f_tol=F_TOL):
    """Compare GPU trace records (dicts) with the oracle's IterRecords until
    the first discrete divergence; returns the number of iterates compared."""
    n = 0
    for a, b in zip(trace, ref_trace):
        assert abs(a["f"] - b.f) <= f_tol * half, f"{what} it {b.it}: f {a['f']} vs {b.f}"
        assert abs(a["rho"] - b.rho) <= RHO_REL * b.rho + RHO_ABS, \
            f"{what} it {b.it}: rho {a['rho']} vs {b.rho}"
        n += 1
        if a["restart"] != b.restart or a["m"] != b.m or a["nfev"] != b.nfev:
            break
        if b.nfev:
            assert abs(a["beta"] - b.beta) <= BETA_REL * max(1.0, abs(b.beta)), \
                f"{what} it {b.it}: beta {a['beta']} vs {b.beta}"
    return n
