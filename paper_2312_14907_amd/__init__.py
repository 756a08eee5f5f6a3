"""MI355X (gfx950) library for the multi-peak Bragg ptychography objective and gradient.

The compute lives in libmpbp.so (C-ABI in include/mpbp.h, HIP kernels in csrc/); this
package holds the build script, the ctypes binding and the torch.autograd wrapper.
Importing `binding` (or any name below) loads the library and fails loudly if it has
not been built.
"""

__all__ = ["Plan", "MPBPError", "MPBPLoss", "binding", "autograd"]


def __getattr__(name):
    # importlib, not "from . import x": the latter asks this module for the attribute
    # first and would recurse into __getattr__ before the submodule is loaded
    import importlib
    if name in ("Plan", "MPBPError", "binding"):
        binding = importlib.import_module(__name__ + ".binding")
        return binding if name == "binding" else getattr(binding, name)
    if name in ("MPBPLoss", "autograd"):
        autograd = importlib.import_module(__name__ + ".autograd")
        return autograd if name == "autograd" else autograd.MPBPLoss
    raise AttributeError(name)
