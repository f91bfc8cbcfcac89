"""MI355X (gfx950) library for canonical tensor decomposition by ALS
accelerated with nonlinear GMRES.

The compute path is the shared library ``libcpng.so`` (HIP kernels for
gfx950 behind the C ABI in include/cpng.h); this package only marshals torch
device tensors into its calls.  Names follow the C ABI.
"""
from ._native import (  # noqa: F401
    CpError, Handle, NGMRESState, PREC, Tensor, cp_als_sweep, cp_decompose, cp_gram,
    cp_mttkrp, cp_mttkrp_noalloc, cp_mode_solve, cp_normalize, cp_objective_grad, cp_tensor_prepare, cp_tensor_release,
    iterate_length, lib, ngmres_accelerate, ngmres_step, options, LIB_PATH, cp_profile,
    cp_profile_read, cp_profile_select, CP_KERNEL_DENSE_MTTKRP, CP_KERNEL_SPARSE_MTTKRP, CP_KERNEL_STREAM_READ,
    CP_KERNEL_GROUP_MTTKRP, CP_KERNEL_DENSE_MTTKRP_F64, CP_KERNEL_SPARSE_GATHER, CP_KERNEL_DENSE_TWOSIDED,
    CP_KERNEL_DENSE_TWOSIDED_F64, cp_stream_read, cp_sparse_gather_read, cp_batch_decompose, Server, cp_init_uniform,
)
