"""MI355X-native matrix repartitioning + Jacobi-PCG (HIP library librp.so).

Importing the package loads the HIP library; it raises ImportError when
librp.so has not been built.  There is no CPU fallback.
"""
from .rp import (Plan, RpError, default_opts, library_path, rcm_order, RP_OK, RP_NOT_CONVERGED, RP_ERR_ARG,
                 RP_ERR_MESH, RP_ERR_OVERFLOW, RP_ERR_HIP, RP_ERR_UNSUPPORTED, RP_ERR_BREAKDOWN,
                 RP_ERR_VALUE, RP_FP64, RP_MIXED, RP_FP32, RP_MIXED_RR, RP_CG, RP_BICGSTAB, RP_KERNEL_SPMV64,
                 RP_KERNEL_SPMV32, RP_KERNEL_SCATTER, RP_LOOP_AUTO, RP_LOOP_COOPERATIVE, RP_LOOP_THREE,
                 RP_LOOP_TWO_MAX_ROWS)

__all__ = ["Plan", "RpError", "default_opts", "library_path", "rcm_order", "RP_OK", "RP_NOT_CONVERGED", "RP_ERR_ARG",
           "RP_ERR_MESH", "RP_ERR_OVERFLOW", "RP_ERR_HIP", "RP_ERR_UNSUPPORTED", "RP_ERR_BREAKDOWN",
           "RP_ERR_VALUE", "RP_FP64", "RP_MIXED", "RP_FP32", "RP_MIXED_RR", "RP_CG", "RP_BICGSTAB",
           "RP_KERNEL_SPMV64", "RP_KERNEL_SPMV32", "RP_KERNEL_SCATTER", "RP_LOOP_AUTO", "RP_LOOP_COOPERATIVE",
           "RP_LOOP_THREE", "RP_LOOP_TWO_MAX_ROWS"]
