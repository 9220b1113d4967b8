"""MI355X (gfx950) implementation of the Dual Natural Gradient Descent step.

The compute lives in libdngd.so (HIP kernels behind the C ABI of
include/dngd.h); ``paper_2505_21404_amd.dngd`` is the ctypes binding,
``driver`` the D-NGD training loop, ``autograd`` the torch.autograd.Function
of the residual map, ``serving`` the continuous-batching job loop.
Importing ``dngd`` without a built library raises ImportError.
"""
import importlib

__all__ = ["dngd", "driver", "autograd", "serving", "build"]


def __getattr__(name):
    if name in __all__:
        return importlib.import_module(f"{__name__}.{name}")
    raise AttributeError(name)
