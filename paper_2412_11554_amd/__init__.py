"""MI355X (gfx950) ACCORD-FBS: HIP kernels behind a C ABI (include/accord.h).

Submodules:
  accord  -- ctypes binding with the C entry-point names (loads libaccord.so)
  build   -- compiles libaccord.so in-tree with hipcc
The binding is imported lazily so that importing the package needs no GPU.
"""
__all__ = ["accord", "build"]
