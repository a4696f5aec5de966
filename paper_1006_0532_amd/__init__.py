"""MI355X-native particle time step of the non-hybrid PDF method on unstructured grids.

The compute path is ``libpdfgpu.so`` (hand-written HIP for gfx950 behind a C ABI,
declared in ``include/pdf.h``).  ``pdfgpu`` is its thin ctypes binding;
``workloads`` generates seeded synthetic meshes and nodal fields.  Nothing is
loaded at import time, so the package imports on machines without a GPU.
"""
__all__ = ["workloads", "pdfgpu"]
