"""MI355X-native QPT-assisted MPDO simulator (arXiv 2508.07610).

Submodules:
  mpdo       -- ctypes binding of libmpdo.so (the C ABI in include/mpdo.h)
  workloads  -- seeded synthetic inputs (gates, channels, circuits, graphs)
  build      -- hipcc build of libmpdo.so for gfx950
Importing the package loads nothing; ``paper_2508_07610_amd.mpdo.lib()``
loads the shared library and raises if it has not been built.
"""
__all__ = ["mpdo", "workloads", "build"]
