"""MI355X-native IPCS (incremental pressure-correction) step for the
incompressible Navier-Stokes equations with Taylor-Hood P2-P1 elements.

The solver is the C-ABI library lib/libipcs.so (HIP kernels for gfx950,
declared in include/ipcs.h); `paper_2605_25403_amd.ipcs` is its ctypes
binding. Importing this package does not load the library; importing
`paper_2605_25403_amd.ipcs` does, and fails if it is not built.
"""
