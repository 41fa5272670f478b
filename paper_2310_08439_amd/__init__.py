"""TensorMD energy/force evaluation on MI355X (gfx950): HIP kernels behind a C ABI.

Submodules:
  inputs  -- seeded synthetic lattices, species, velocities and MLP weights
  tmd     -- ctypes binding of libtmd.so (device pointers from torch tensors)
  build   -- hipcc build of libtmd.so
"""
