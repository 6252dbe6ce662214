"""MI355X-native phonon BTE time step (HIP kernels behind a C ABI).

Submodules:
  inputs -- seeded synthetic problem instances (no solver arithmetic)
  bte    -- ctypes binding of libbte.so (include/bte.h); needs the built library
  build  -- hipcc build of libbte.so for gfx950
"""
__all__ = ["inputs", "bte", "build"]
