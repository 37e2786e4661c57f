"""WENOIU schemes with free-stream preservation on MI355X (gfx950).

Submodules:
  wenoiu     -- ctypes binding of libwenoiu.so (include/wenoiu.h); needs the
                built library and a ROCm device for every compute call.
  workloads  -- seeded synthetic grids and initial states (inputs only).
  build      -- in-tree hipcc build of libwenoiu.so.
"""
