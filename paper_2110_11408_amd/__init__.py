"""MI355X-native CompaSO halo finding (HIP library libhf + a thin Python binding).

Submodules:
  api    -- Context with density / l0_fof / compaso / find on torch GPU tensors
  _lib   -- ctypes declarations of the C ABI (include/hf.h)
  synth  -- seeded synthetic particle boxes (inputs only)
  build  -- hipcc build of libhf.so
"""
