"""MI355X (gfx950) mixed-precision HODLR matrix-vector product.

The product Y = A_H X of Carson, Chen, Liu, "Mixed Precision HODLR Matrices"
(arXiv 2407.21637) runs in hand-written HIP kernels behind the C ABI of
``include/hodlr.h`` (built into ``libhodlr.so`` by ``build.py``).  This
package only marshals arguments to that library; PyTorch supplies device
memory and streams.
"""
from ._lib import (ACC_FP32, ACC_FP64, DTYPES, EXPORTS, KERNELS, NO_COLUMN_SCALE, PER_BLOCK, HodlrError, Operator,
                   build_kernel, colmajor_empty, depth_for_leaf, lib, matvec_batched, tree_blocks, tree_bounds)

__all__ = ["ACC_FP32", "ACC_FP64", "DTYPES", "EXPORTS", "KERNELS", "NO_COLUMN_SCALE", "PER_BLOCK", "HodlrError",
           "Operator", "build_kernel", "colmajor_empty", "depth_for_leaf", "lib", "matvec_batched", "tree_blocks",
           "tree_bounds"]
