"""Lyman-alpha mock hot path (arXiv 2310.18996) for AMD MI355X.

The compute lives in liblyamock.so (HIP, gfx950; C-ABI in include/lyamock.h);
`lyamock` is its ctypes binding.
"""
from . import lyamock  # noqa: F401

__all__ = ["lyamock"]
