"""MI355X (gfx950) grand-canonical Monte Carlo cell-list hot path.

The method is Schwiebert et al., "An Efficient Cell List Implementation for
Monte Carlo Simulation on GPUs" (arXiv 1408.3764).  The product is the C-ABI
library ``libgcmc.so`` (``include/gcmc.h``), hand-written HIP for gfx950; this
package is its thin Python binding:

* ``_lib``       ctypes binding, one function per C entry point (same names)
* ``box``        Box / Batch handles (marshalling numpy/torch <-> C ABI)
* ``autograd``   torch.autograd.Function over total energy and its gradient
* ``tune``       the autotuner of launch shapes and cell sizes
* ``workloads``  seeded synthetic inputs shaped like the paper's workloads
* ``build``      hipcc build of libgcmc.so

Importing the package does not load the library; the first call does, and
raises if it is not built (there is no CPU fallback).
"""

__all__ = ["Box", "Batch", "make_moves", "workloads"]


def __getattr__(name):
    if name in ("Box", "Batch", "make_moves"):
        from . import box as _box
        return getattr(_box, name)
    raise AttributeError(name)
