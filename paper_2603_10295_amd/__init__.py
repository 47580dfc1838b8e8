"""MI355X-native Wannier-to-Bloch interpolation of electron-phonon matrix elements.

The computation lives in the HIP library ``libephw.so`` (C ABI in
``include/ephw.h``); ``ephw`` is its ctypes binding, ``autograd`` wraps the
loss and its adjoint as a torch.autograd.Function, and ``model`` holds the
host-side cost and size accounting used for reporting.
"""
from . import ephw, model  # noqa: F401

__all__ = ["ephw", "model", "autograd"]
