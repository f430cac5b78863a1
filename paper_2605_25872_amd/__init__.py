"""PTHR on MI355X: Parallel Tempering with Houdayer all-cluster moves and an
entropic Reservoir for the 3D Gaussian Edwards-Anderson spin glass, as HIP
kernels for gfx950 behind a C ABI (include/pthr.h).

``pthr.Pthr`` is the Python binding; ``inputs`` generates seeded couplings and
temperature grids; ``build`` compiles ``libpthr.so`` in-tree.
"""
