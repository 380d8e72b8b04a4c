"""MI355X (gfx950) exhaustive AND/OR traversal of metabolic networks.

Modules:
  netgen  seeded synthetic networks (input data only)
  efm     ctypes binding of libefm.so (include/efm.h)
  build   hipcc build of libefm.so
"""
