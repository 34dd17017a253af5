"""MI355X-native particle-in-cell Boltzmann step (arXiv:1208.0961, CuBA).

The compute path lives in the HIP library libcuba.so (csrc/); the Python
side only marshals arguments through ctypes (``paper_1208_0961_amd.cuba``)
and draws synthetic inputs (``paper_1208_0961_amd.workload``).  Importing
the package loads nothing; ``paper_1208_0961_amd.cuba`` loads the library
and raises if it is missing.
"""
__all__ = ["cuba", "workload"]
