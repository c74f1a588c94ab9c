"""MI355X G1-G2 propagator: HIP kernels behind a C ABI (include/g1g2.h) and a
thin ctypes binding.  Import ``binding`` for the calls; ``build.build()``
compiles the library in-tree for gfx950."""
