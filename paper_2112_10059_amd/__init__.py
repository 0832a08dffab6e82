"""MI355X-native adaptive fast-multipole photoionization (Lin & Zhuang, arXiv 2112.10059).

The product is libph.so (HIP kernels for gfx950 behind the C ABI in include/ph.h);
``binding`` is its thin ctypes wrapper.
"""
from . import binding  # noqa: F401
