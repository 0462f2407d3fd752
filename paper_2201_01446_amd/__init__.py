"""Compressed Deep Potential force step on MI355X (gfx950).

The computation lives in libdp.so (hand-written HIP kernels behind the C-ABI
of include/dp.h).  This package is the thin Python side: `Model`,
`NeighborList`, `compute`, `nve_run`, `nve_continue`, the autograd function in
`autograd`, and the serving loop in `serve`.  PyTorch provides device memory
and streams only.
"""
from .api import (COMPRESSED, FP32, FP64, FUSED, FUSED_PADDED, MIXED_BF16, PLAIN, TAB_UNFUSED, DPError,  # noqa: F401
                  Model, NeighborList, compute, descriptor, nve_continue, nve_run)
