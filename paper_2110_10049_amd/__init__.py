"""GOSH hot path on MI355X (gfx950): MultiEdgeCollapse coarsening, TrainInGPU
training and copy prolongation behind the C ABI of include/gosh.h.

``gosh`` is the ctypes binding of libgosh.so; ``driver`` runs Algorithm 2 over
it.  Build the library with ``paper_2110_10049_amd.build.build()``.
"""
