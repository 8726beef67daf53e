"""MI355X (gfx950) variable-coefficient MAC projection by geometric multigrid.

Submodules:
  inputs   -- seeded synthetic problems (no projection arithmetic)
  macproj  -- ctypes binding of the HIP library libmacproj.so
  build    -- hipcc build of the library
"""
