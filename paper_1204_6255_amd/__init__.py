"""MI355X (gfx950) D-iteration: DI-SOP fluid diffusion for X = P.X + B.

Submodules:
  di        ctypes binding of libdi (the C ABI in include/di.h)
  graphgen  seeded synthetic web-graph inputs and Table-1 statistics
  build     builds libdi.so (hipcc) and libdigen.so (g++) in-tree

Nothing is loaded at import time; libdi is opened on first use.
"""

__all__ = ["di", "graphgen"]
