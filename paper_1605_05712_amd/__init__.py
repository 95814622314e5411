"""MI355X-native generalized Basic Scheme on lattice patterns.

The computation lives in libahom.so (HIP for gfx950, C ABI declared in
include/ahom.h); ``paper_1605_05712_amd.ahom`` is its ctypes binding.
"""
