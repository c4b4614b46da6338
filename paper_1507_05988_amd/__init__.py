"""MI355X (gfx950) implementation of the 2D+1 split-step Fourier / Crank-Nicholson z-step
of Ma & Lin (arXiv:1507.05988).

Modules: ``fcn`` (binding of the C ABI in include/fcn.h; the HIP kernels do all the
work), ``workloads`` (seeded synthetic pulses), ``build`` (hipcc build of libfcn.so).
Importing the package loads nothing; ``fcn.load_library()`` raises when the library is
missing, and ``fcn.Plan`` raises without a GPU.
"""
__all__ = ["fcn", "workloads", "build"]
