"""MI355X (gfx950) HIP implementation of the mixed half-range / full-range Gauss-Hermite
lattice Boltzmann time step for 3D Couette flow with the Shakhov collision term
(Ambrus & Sofonea, arXiv:1702.01335).

The solver lives in the C-ABI library libhrlb.so (include/hrlb.h); ``hrlb`` is its
Python binding, ``inputs`` the seeded input generator, ``workloads`` the named
parameter sets.  Build with ``python -m paper_1702_01335_amd.build``.
"""
