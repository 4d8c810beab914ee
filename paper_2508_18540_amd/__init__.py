"""MI355X sweeping-plane light-field renderer: Python side of the C ABI in ``include/lf.h``.

``_lib`` is the ctypes binding (one Python function per C entry point);
``torch_api`` marshals torch CUDA tensors into those calls.  All compute runs in
the HIP kernels of ``liblf.so``; importing ``torch_api`` without the built library
raises ImportError.
"""
from . import _lib  # noqa: F401
from ._lib import LFError  # noqa: F401
