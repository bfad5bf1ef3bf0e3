"""MI355X-native integer sorting (arXiv 1808.10292 hot path): HIP kernels for
gfx950 behind the C ABI in include/rsort.h, with a ctypes binding.

The binding module (``paper_1808_10292_amd.rsort``) is imported lazily so that
``import paper_1808_10292_amd.build`` works without torch or a built library.
"""
import importlib

__all__ = ["rsort"]


def __getattr__(name):
    if name == "rsort":
        return importlib.import_module(__name__ + ".rsort")
    raise AttributeError(name)
