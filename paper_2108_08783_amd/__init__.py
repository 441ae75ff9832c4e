"""MI355X-native elastic-wall D3Q19 lattice Boltzmann (McCullough & Coveney).

The compute path is the HIP library ``liblbm.so`` built from ``csrc/``;
``lbm`` is its ctypes binding.  Importing this package loads nothing: the
library is opened on first use of ``paper_2108_08783_amd.lbm``.
"""
__all__ = ["inputs", "lbm"]
