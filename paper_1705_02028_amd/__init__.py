"""MI355X-native residual-distribution hot path (N / LDA / B schemes, RK2)
for the two-dimensional Euler equations on triangular meshes.

``paper_1705_02028_amd.rd`` is the Python binding of the C-ABI library
``librd.so`` (HIP kernels for gfx950); ``paper_1705_02028_amd.inputs`` builds
seeded synthetic meshes and initial states. Importing the package loads
nothing: the binding loads the library on first use and raises if it is
missing.
"""
