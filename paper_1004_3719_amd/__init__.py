"""Exact sparse matrix products over Z/mZ on MI355X (gfx950).

The compute path is libffx.so (hand-written HIP kernels behind the C ABI of
include/ffx.h); `ffx` is its ctypes binding. Importing this package does not
load the library; the first call does, and raises if it was not built.
"""
from .ffx import (FORMATS, Batch, FfxError, Matrix, Selector, block_features, build_opts, check_block,  # noqa: F401
                  lib, reorder_rcm, sequence_rank, set_sequence_graph_batch, sigma_basis, version)

__all__ = ["Matrix", "Batch", "Selector", "FfxError", "FORMATS", "block_features", "build_opts", "lib",
           "set_sequence_graph_batch", "check_block", "reorder_rcm", "sigma_basis", "sequence_rank", "version"]
