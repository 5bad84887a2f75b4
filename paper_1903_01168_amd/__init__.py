"""MI355X-native two-population colour-gradient lattice Boltzmann (D2Q9).

The method (arXiv:1903.01168, Sec. 2) runs in hand-written HIP kernels behind
the C ABI of ``include/cglbm.h`` (``libcglbm.so``); :mod:`.capi` is the thin
ctypes binding and :mod:`.workloads` the seeded synthetic inputs.  Importing
the package does not load the library; :func:`capi.load` does, and fails
loudly when it has not been built.
"""
__all__ = ["capi", "workloads"]
