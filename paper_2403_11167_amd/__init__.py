"""MI355X-native D2Q9 multiphase lattice Boltzmann library (pseudopotential
and well-balanced free-energy models of Czelusniak et al., arXiv 2403.11167).

The compute path is the HIP library ``liblbm.so`` behind the C ABI declared
in ``include/lbm.h``; :mod:`paper_2403_11167_amd.lbm` is its thin ctypes
binding.  Importing this package does not load the library.
"""
__all__ = ["lbm", "inputs"]
