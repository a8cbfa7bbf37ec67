"""VOctree rendering for MI355X (gfx950): the rendering hot path of NeuVV
(arXiv 2202.06088) as hand-written HIP kernels behind a C ABI
(include/neuvv.h, libneuvv.so), with a thin Python binding.

Modules: _lib (ctypes binding, same names as the C ABI), voctree (tree
container), ops (functional calls, including the shadow-map low-pass and the
lighting pass), autograd (RenderFn, ComposeFn), build (hipcc build of
libneuvv.so).
"""
from . import _lib  # noqa: F401
from ._lib import BF16, F16, F32, NeuvvError, make_camera, make_instance, make_light  # noqa: F401

__all__ = ["F32", "F16", "BF16", "NeuvvError", "make_camera", "make_instance", "make_light", "load"]


def load():
    """Loads libneuvv.so; raises ImportError when it has not been built."""
    return _lib.load()
