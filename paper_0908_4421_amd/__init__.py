"""MI355X (gfx950) fluence-map optimiser: gradient projection with Armijo's
line search over a CSR/CSC dose-deposition matrix (arXiv:0908.4421).

The compute path is libimrt.so (HIP kernels behind a C ABI, include/imrt.h);
``paper_0908_4421_amd.imrt`` is its ctypes binding.
"""
from . import imrt  # noqa: F401

__all__ = ["imrt"]
