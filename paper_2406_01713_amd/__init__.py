"""Walk-on-Spheres estimates of screened-Poisson potential fields on MI355X.

Modules:
    scenes    seeded synthetic workloads (inputs only)
    binding   ctypes binding of libwos.so, the HIP library (import raises if
              the library is not built: there is no CPU fallback)
    autograd  torch.autograd.Function over wos_estimate / wos_backward
    build     hipcc build of libwos.so for gfx950
"""
__all__ = ["scenes", "binding", "autograd", "build"]
