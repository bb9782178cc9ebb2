"""MI355X-native superpixel-plane matching cost for sparse light fields.

The compute path is the HIP library libslf.so (C ABI in include/slf.h);
paper_1812_06856_amd.slf is its Python binding.
"""
from . import build  # noqa: F401


def context(device: int = 0):
    from .slf import Context

    return Context(device)
