"""MI355X-native batched Paillier hot path of the 3P-ADMM-PC2 method.

The product is ``libpc2.so`` (HIP kernels for gfx950 behind the C ABI in
``include/pc2.h``); ``paper_2601_14980_amd.pc2`` is its thin Python binding.
Submodules are imported lazily so that ``build`` works before the library
exists.
"""

__all__ = ["pc2", "build"]
