"""MI355X (gfx950) implementation of the synchronous quantum-inspired
low-energy search for fully connected Ising Hamiltonians (arXiv:2010.00180).

Submodules:
  binding    ctypes access to the HIP library (include/ising_search.h)
  workloads  seeded synthetic instances (no method arithmetic)
  build      compiles the HIP library in-tree with hipcc for gfx950
"""
__all__ = ["binding", "workloads", "build"]
