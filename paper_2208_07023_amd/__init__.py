"""MI355X-native per-node split search of the accelerated Subspace Learning
Machine (Fu et al., arXiv 2208.07023).

The compute path is the HIP library `libslm.so` (C ABI declared in
include/slm.h); `api` is its thin Python binding over torch device tensors and
`inputs` holds the seeded synthetic input generators.
"""
__all__ = ["api", "inputs"]
