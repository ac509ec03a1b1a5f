"""MI355X-native (gfx950) moving-body lattice kinetic scheme: forward sweep, rigid-body grid
transfer and exact discrete adjoint behind the C ABI of include/lks.h.

Submodules: ``lks`` (ctypes binding of liblks.so), ``autograd`` (torch.autograd.Function),
``server`` (continuous-batching sensitivity server), ``build`` (hipcc build of liblks.so).
"""
__all__ = ["lks", "build"]
