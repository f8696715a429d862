"""MI355X-native cell-centred Lagrangian ADER-MOOD step for neo-Hookean
solids (Boscheri, Loubere & Maire, arXiv 2104.02139).

The compute path is the HIP library ``libhyperlag.so`` (C-ABI declared in
``include/hyperlag.h``); ``paper_2104_02139_amd.hyperlag`` is its ctypes
binding.  Nothing is imported eagerly so that input generation works on a
machine without the library.
"""
__all__ = ["hyperlag", "workloads"]
