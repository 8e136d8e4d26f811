"""MI355X (gfx950) implementation of the Toeplitz MBIR hot path of arXiv 2603.28756.

The compute lives in ``lib/libtomo.so`` (HIP kernels behind the C ABI of
``include/tomo.h``); ``paper_2603_28756_amd.tomo`` is its ctypes binding and
``paper_2603_28756_amd.build`` compiles it.  Importing this package does not
load the library; the first binding call does, and raises if it is missing.
"""
__all__ = ["build", "tomo"]
