"""MI355X-native TENO5-LAD Euler right-hand side (Peng et al., arXiv:2003.09145).

The numerical path runs in hand-written HIP kernels for gfx950 behind the
C-ABI library ``libteno.so`` (declared in ``include/teno.h``).  This package is
the thin Python binding over that library (argument marshalling only) plus the
seeded input generators in :mod:`.workloads`.  Importing the package does not
load the GPU library; the first call into :mod:`.binding` does, and fails
loudly if it is missing.
"""
__all__ = ["binding", "workloads"]
