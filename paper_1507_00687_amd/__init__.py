"""MI355X-native recursive bilinear fast matrix multiplication (arXiv 1507.00687).

The computation runs in libfastmm.so (hand-written HIP kernels for gfx950) behind the C ABI
declared in include/fastmm.h; this package is a thin binding over it.
"""
from .autograd import FastMatmulFn, fast_matmul  # noqa: F401
from .fastmm import (  # noqa: F401
    ALGOS,
    PRECISIONS,
    SCALE_MODES,
    FastmmError,
    Plan,
    fastmm_algo_coeffs,
    fastmm_algo_info,
    fastmm_algo_register,
    fastmm_algo_stability,
    fastmm_batched_workspace_size,
    fastmm_gemm,
    fastmm_gemm_backward,
    fastmm_gemm_backward_batched,
    fastmm_gemm_batched,
    fastmm_gemm_batched_ex,
    fastmm_gemm_ex,
    fastmm_gemm_noalloc,
    fastmm_profile_enable,
    fastmm_profile_read,
    fastmm_scaling_exponents,
    fastmm_task_table,
    lib,
    matmul,
)
