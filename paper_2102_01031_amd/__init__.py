"""MI355X-native lattice field step (CosmoLattice method, arXiv:2102.01031).

The compute path is the HIP library ``csrc/liblattice.so`` behind the C ABI of
``include/lattice.h``; ``lattice`` is its thin ctypes binding.  Importing this
package loads nothing; the binding loads the library on first use and raises
if it is missing.
"""
__all__ = ["inputs", "workloads", "lattice"]
