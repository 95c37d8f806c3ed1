"""MI355X-native accelerated spherical k-means (libskm).

The product is the C-ABI library ``lib/libskm.so`` built from ``csrc/``
(hand-written HIP for gfx950); ``skm`` is its thin ctypes binding.
Importing this package loads nothing; ``skm.load()`` does, and fails loudly
when the library has not been built.
"""
__all__ = ["skm", "build"]
