"""Serial FP64 oracle of the repartitioning path (test infrastructure only).

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package.  The product library never uses it, and it shares no
code with the GPU path.
"""
from .oracle import (OracleError, Merged, build, loaded_library, merge, receive_buffer,
                     update, spmv, pcg, bicgstab, bicgstab_csr, true_relres, value_grad, face_grad,
                     block_starts, block_jacobi_inverse, block_jacobi_apply, pcg_block_jacobi, AmgHierarchy)

__all__ = ["OracleError", "Merged", "build", "loaded_library", "merge", "receive_buffer",
           "update", "spmv", "pcg", "bicgstab", "bicgstab_csr", "true_relres", "value_grad", "face_grad",
           "block_starts", "block_jacobi_inverse", "block_jacobi_apply", "pcg_block_jacobi", "AmgHierarchy"]
