"""MI355X (gfx950) implementation of the global low-rank (GLR) prior step
(arXiv 2301.03047) behind the C ABI of ``include/glr.h``.

``Plan`` is a thin ctypes binding: it marshals torch device tensors and the
current HIP stream into the library calls; every step runs in the library's
HIP kernels.  Importing works without a GPU; calls need the built
``libglr.so`` and a device.
"""
from .glr import (Plan, Cnn, GlrError, lib, library_path, CACTI, MRI, MSFA,
                  STATUS_NAMES, STATIC_SCRATCH_BYTES)

__all__ = ["Plan", "Cnn", "GlrError", "lib", "library_path", "CACTI", "MRI", "MSFA", "STATUS_NAMES",
           "STATIC_SCRATCH_BYTES"]
