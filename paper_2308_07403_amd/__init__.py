"""MI355X (gfx950) engine for the R-distance all-pairs shortest paths of
Jing & Meister (arXiv 2308.07403).

The compute lives in ``librdist.so`` (HIP kernels behind the C ABI of
``include/rdist.h``); ``paper_2308_07403_amd.rdist`` is its ctypes binding.
Importing the binding raises if the library has not been built.
"""
__all__ = ["rdist"]
