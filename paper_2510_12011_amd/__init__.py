"""MI355X-native hot path of the monodomain finite-element method of TorchCor
(arXiv 2510.12011): ionic update, theta-method right-hand side and
Jacobi-preconditioned CG over a P1 tetrahedral mesh, as hand-written HIP
kernels for gfx950 behind a C ABI (include/monox.h).

Submodules: ``inputs`` (seeded synthetic meshes and run descriptions),
``_lib`` (ctypes binding of libmonox.so), ``sim`` (Python front end that
gives the library torch-allocated device memory and the torch stream),
``build`` (hipcc build of libmonox.so).
"""
__all__ = ["inputs", "sim", "build"]
