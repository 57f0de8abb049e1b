"""MI355X (gfx950) incident-wave hot path of the two-phase SWENSE method:
HOS free-surface step, modal evaluation on an intermediate grid, and
interpolation to CFD cell centres, behind the C ABI of include/swense.h.

The compute lives in libswense.so (hand-written HIP); `lib` is the ctypes
binding.  Importing this package does not load the library; lib.load() does
and raises if it has not been built.
"""
__all__ = ["lib"]
