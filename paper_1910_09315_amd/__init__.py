"""MI355X (gfx950) overset grid assembly: hole cutting, fringe compaction,
query transform, donor search and trilinear interpolation as hand-written
HIP kernels behind a C ABI (include/overset.h).

Importing the package loads nothing; `binding.load()` loads liboverset.so
and raises if it has not been built.
"""
__all__ = ["binding", "assembly", "build"]
