"""MI355X-native HSS-ULV: construction, factorization, solve and matvec of
hierarchically semi-separable SPD kernel matrices on one gfx950 GPU.

The compute lives in libhss.so (HIP, C ABI declared in include/hss.h); the
`hss` submodule is its Python binding.
"""
__all__ = ["hss"]
