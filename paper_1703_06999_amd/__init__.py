"""MI355X-native vdW-DF nonlocal correlation (Roman-Perez--Soler form) on one GPU.

Submodules are imported on demand: ``inputs`` (seeded synthetic densities and kernel tables),
``vdwxc`` (the binding of the C-ABI library), ``autograd`` and ``serving``.
"""
__all__ = ["inputs", "vdwxc", "autograd", "serving"]
