"""MI355X (gfx950) batched approximate kNN: the Multicurves search path of
Hypercurves (Teodoro et al., arXiv 1209.0410) as hand-written HIP kernels
behind a C ABI (include/hypercurves.h).

Submodules:
  capi     ctypes binding of libhypercurves.so (same names as the header)
  index    Index / search over device tensors
  datagen  seeded synthetic inputs (random numbers only)

Importing the package loads nothing; the library is loaded on first use and
its absence is an error (there is no CPU fallback).
"""
