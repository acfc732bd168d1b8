"""MI355X map-making: block-Jacobi PCG for (P^T N^-1 P) m = P^T N^-1 d on one GPU.

The computation lives in the HIP library ``libmm.so`` (sources in ``csrc/``, ABI in
``include/mm.h``); ``mapmaker`` is its ctypes binding.
"""

__all__ = ["mapmaker", "build"]
