"""MI355X-native expectation propagation for 3-D Gaussian-process extinction
mapping (after Sale & Magorrian, arXiv:1708.09705).

The numerical work lives in the HIP library ``libep.so`` (csrc/, C ABI in
include/ep.h); ``paper_1708_09705_amd.ep`` is its Python binding.
"""
