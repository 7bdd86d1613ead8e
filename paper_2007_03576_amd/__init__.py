"""MI355X-native multishift QR with aggressive early deflation (Hessenberg -> real Schur form).

Python side of libhqr.so: every step of the computation runs in the library's
HIP kernels; this package only marshals torch device tensors and streams.
"""
from .api import (BatchedGraph, BatchedProblem, HqrError, batched_launch, eigenvectors, eigvals, hessenberg,
                  last_stats, params, schur, schur_batched, schur_colmajor, set_batched_launch, set_params,
                  set_batched_table, batched_table, qz_batched)

__all__ = ["schur", "schur_colmajor", "schur_batched", "eigvals", "hessenberg", "eigenvectors", "set_params", "params",
           "set_batched_table", "batched_table",
           "last_stats", "HqrError", "BatchedProblem", "BatchedGraph", "set_batched_launch",
           "batched_launch", "qz_batched"]
