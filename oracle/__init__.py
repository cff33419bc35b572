"""CPU oracle for compressed contraction-tree execution — TEST INFRASTRUCTURE ONLY.

Plain, slow, float64 numpy implementations of what the GPU library computes,
written from the paper (Gray & Chan, arXiv:2206.07044) and sharing no code
with the library: ``approx`` is Algorithm 1 (section II.F) with QR-reduced
bond compression (section II.C, Eq. (svd)) and the projector form (SI B);
``exact`` holds independent exact references (brute force, transfer
matrices, matching counts) used to pin it; ``grad`` is the reverse-mode
adjoint of the same forward pass (textbook truncated-SVD adjoint over the
complete core spectrum), the reference gradient; ``projnet`` builds the explicit
projector network T_P of SI B from an oracle run (its exact contraction equals the
compressed value).

Only tests, the smoke check and the benchmark's CPU-baseline leg may import
this package.  The library never calls it and has no fallback to it.
"""
from .approx import contract_compressed, OracleResult, OpRecord
from . import exact, grad

__all__ = ["contract_compressed", "OracleResult", "OpRecord", "exact", "grad"]
