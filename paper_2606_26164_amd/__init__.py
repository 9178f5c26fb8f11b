"""MI355X-native ChiSao per-cycle population update (libchisao + a thin binding).

The HIP library is loaded on first use; importing this package does not need
a GPU.  There is no CPU fallback: every step runs in the library's kernels.
"""
from . import _lib  # noqa: F401

__all__ = ["Optimizer", "log_density", "ChisaoLogDensity"]


def __getattr__(name):
    if name == "Optimizer":
        from .api import Optimizer

        return Optimizer
    if name in ("log_density", "ChisaoLogDensity"):
        from . import autograd

        return getattr(autograd, name)
    raise AttributeError(name)
