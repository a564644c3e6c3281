"""MI355X-native two-phase D2Q9 lattice-Boltzmann step with mass-conservative
curved-wall schemes (Yu, Li & Wen, arXiv:1908.09235).

The compute path is the HIP library ``liblbm2p.so`` (C ABI in
``include/lbm2p.h``); ``paper_1908_09235_amd.lbm`` is its ctypes binding.
Importing this package does not load the library; the binding raises if the
library has not been built (``python -m paper_1908_09235_amd.build``).
"""
__all__ = ["lbm"]
