"""MI355X-native D2Q9 MRT lattice Boltzmann step with the absorbing-layer
damping terms of Xu & Sagaut (arXiv:1203.6350).

The compute path is liblbm.so (HIP, gfx950) behind the C ABI of
include/lbm.h; ``paper_1203_6350_amd.lbm`` is its ctypes binding.
Importing this package loads nothing; the library is loaded on first use.
"""
__all__ = ["lbm", "workloads", "build"]
