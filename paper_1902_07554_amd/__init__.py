"""MI355X-native sample-based divide-and-conquer Delaunay triangulation.

The hot path lives in libdt.so (HIP kernels for gfx950 behind the C ABI in
include/dt.h); `binding` is its thin Python binding and `inputs` holds the
seeded synthetic point-set generators.  Importing the package does not load
the library; the first binding call does, and fails loudly if it is not
built.
"""
__all__ = ["binding", "inputs", "build"]
