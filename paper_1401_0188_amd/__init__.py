"""MI355X-native D2Q13 energy-conserving lattice Boltzmann step (HIP for gfx950).

The compute path is ``csrc/`` (HIP kernels behind the C ABI declared in
``include/lbm13.h``); ``lbm13`` is the thin ctypes binding.  Importing the
package does not load the library; ``paper_1401_0188_amd.lbm13`` does.
"""
__all__ = ["lbm13", "workloads"]
