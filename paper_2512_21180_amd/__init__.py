"""MI355X-native cone-beam projector pair (forward A and its exact transpose).

Submodules:
  workloads  -- seeded geometries and phantoms (inputs only)
  cbct       -- ctypes binding of the C-ABI library libcbct.so (HIP, gfx950)
"""
