"""MI355X-native ADMM micromechanics solver (Zhou & Bhattacharya, arXiv 2010.06697).

The compute path is a C-ABI shared library (``libadmm.so``, HIP kernels for
gfx950) declared in ``include/admm.h``; ``paper_2010_06697_amd.admm`` is its
thin ctypes binding. ``paper_2010_06697_amd.microstructure`` generates the
seeded synthetic inputs. Importing this package loads nothing; the binding
loads the library on first use and raises if it is missing.
"""
__all__ = ["admm", "microstructure"]
