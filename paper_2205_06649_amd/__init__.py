"""MI355X-native space-time domain-decomposed 4D-Var (local cost/gradient engine).

The computation lives in libdd4dvar.so (HIP kernels for gfx950 behind the C
ABI of include/dd4dvar.h).  This package is its thin Python binding:

* ``_lib``        -- ctypes binding, same names as the C ABI;
* ``descriptors`` -- marshalling of a problem into the descriptor structs,
                     and the host-only ``Plan`` (index maps);
* ``context``     -- ``Context``: device buffers and streams from torch;
* ``autograd``    -- ``LocalSweep``: torch.autograd.Function over the sweeps;
* ``build``       -- in-tree build of the library.
"""
from . import _lib  # noqa: F401

__all__ = ["Context", "Plan", "build"]


def __getattr__(name):
    if name == "Context":
        from .context import Context
        return Context
    if name == "Plan":
        from .descriptors import Plan
        return Plan
    if name == "build":
        from .build import build
        return build
    raise AttributeError(name)
