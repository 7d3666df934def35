"""MI355X-native SCMF hot path (arXiv:1711.03828): HIP kernels behind a C ABI.

``soma``  -- ctypes binding of include/soma.h (one Python function per entry point)
``melt``  -- torch-owned buffers and a handle for one melt
``build`` -- compiles ``libsoma_hip.so`` for gfx950
"""
__all__ = ["soma", "melt", "build"]
