"""RAM (Rapid Advection Algorithm on Arbitrary Meshes) on AMD MI355X.

The advection step -- bulk shift by conservative remap, then the residual
upwind step -- runs in the hand-written HIP kernels of ``libram.so`` behind
the C ABI of ``include/ram.h``.  Python submodules:

  _lib       ctypes binding of the C ABI (``Context.ram_shift`` ...)
  autograd   torch.autograd.Function over a checkpointed rollout
  workloads  seeded synthetic inputs
  build      hipcc build step for libram.so
"""
__version__ = "0.1.0"
