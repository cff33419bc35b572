"""MI355X executor for compressed tensor-network contraction trees.

Evaluates Algorithm 1 of Gray & Chan, "Hyper-optimized approximate
contraction of tensor networks with arbitrary geometry" (arXiv:2206.07044),
with early or late compression and local (r = 0) QR-reduced truncated-SVD
bond compression, in hand-written HIP kernels for gfx950 behind the C ABI of
include/tn.h.  This package is the thin Python binding of that library.
"""
from ._capi import (Batch, Context, TNError, load_library, tn_plan_describe, exported_symbols, LIB_PATH, KERNEL_KINDS,
                    GEMM_CLASSES, GEMM_TILES, tn_gemm_tiles_get, tn_gemm_tiles_set, tn_gemm_tune,
                    TN_OK, TN_EINVAL, TN_ESTATE, TN_ENOMEM, TN_EDEVICE, TN_ENUMERIC, TN_ZERO)
from .scoring import TreeScore, TreeScorer
from .projnet import frozen_projector_grad, projector_network

__all__ = ["projector_network", "frozen_projector_grad", "Batch", "Context", "TNError", "load_library", "tn_plan_describe", "exported_symbols", "LIB_PATH", "KERNEL_KINDS",
           "GEMM_CLASSES", "GEMM_TILES", "tn_gemm_tiles_get", "tn_gemm_tiles_set", "tn_gemm_tune",
           "TN_OK", "TN_EINVAL", "TN_ESTATE", "TN_ENOMEM", "TN_EDEVICE", "TN_ENUMERIC", "TN_ZERO",
           "TreeScore", "TreeScorer"]
