"""MI355X-native directional diffusion splitting solver (arXiv 2411.11041).

The solver is the HIP library libadr.so (C ABI in include/adr.h); `adr` is its
ctypes binding.
"""
from .adr import Solver, ADRError, load  # noqa: F401
