"""MI355X-native fused lattice-Boltzmann step with the enhanced single-node
(ELIBB) boundary condition of arXiv 2009.04604.

Modules:
  binding    ctypes binding of liblbm.so (the C-ABI in include/lbm.h)
  workloads  builds the benchmark workloads (geometry via the library's host
             builder, domains on the GPU)
  build      compiles liblbm.so for gfx950 in-tree
"""
__all__ = ["binding", "workloads", "build"]
