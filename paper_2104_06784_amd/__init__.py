"""MI355X-native two-phase (grain + fluid) shallow-flow step of MoSES_2PDF.

The step runs in hand-written HIP kernels for gfx950 behind the C ABI of
``include/m2p.h`` (``libm2p.so``); this package holds the ctypes binding
(``_abi``, ``sim``), the build script (``build_lib``) and the seeded synthetic
input generators (``inputs``).  Importing the package loads nothing: the
library is opened on first use and the import fails loudly if it was not
built.
"""

__all__ = ["inputs", "sim", "build_lib"]
