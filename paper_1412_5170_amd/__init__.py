"""MI355X-native pseudo-potential D2Q9 lattice Boltzmann (Hu, Li & Uddin, arXiv:1412.5170).

The time step runs in hand-written HIP kernels for gfx950 behind a C ABI
(``include/pplbm.h``, ``libpplbm.so``); ``paper_1412_5170_amd.lbm`` is the thin ctypes
binding with the same function names.  ``paper_1412_5170_amd.inputs`` holds the seeded
synthetic workloads (initial density fields and batch draws) and no arithmetic of the method.
"""

__all__ = ["lbm", "inputs"]
