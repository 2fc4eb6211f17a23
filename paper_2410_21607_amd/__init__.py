"""MI355X spectral-element right-hand side for adaptive tropical-cyclone
simulation (arXiv 2410.21607): HIP kernels behind a C ABI (``libsem.so``,
declared in ``include/sem.h``) and a thin ctypes binding.

Everything on the hot path runs in the HIP library; importing the binding
does not require a GPU, but every compute call does and fails loudly if the
library is missing.
"""

from . import native  # noqa: F401

__all__ = ["native", "api", "solver"]
