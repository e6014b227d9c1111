"""MI355X-native randomized graph propagation (Approximate Graph Propagation,
Wang et al., KDD'21): the level-by-level residue push of Algorithm 2 as HIP
kernels for gfx950 behind the C ABI of include/agp.h.

Submodules:
    agp     ctypes binding of libagp.so (argument marshalling only)
    inputs  seeded synthetic graphs, signals and weight sequences
    build   compiles libagp.so with hipcc
"""
