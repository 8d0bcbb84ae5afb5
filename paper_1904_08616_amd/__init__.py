"""MI355X-native Wilson-Dirac operator (eq. (1)) and CG on D^dagger D
(Algorithm 1) of arXiv:1904.08616, on hand-written HIP kernels for gfx950.

The compute path is libdirac.so (C ABI in include/dirac.h); the submodule
``dirac`` is a thin PyTorch binding of it (``from paper_1904_08616_amd import
dirac``).  Importing this package does not load the library; the first call
does, and fails loudly if it has not been built.
"""

from . import _abi  # noqa: F401
