"""MI355X-native four-step learned-wavelet decode path (pWave++ context model).

The compute lives in libwv.so (HIP kernels for gfx950 behind the C ABI in
include/wv.h); `codec` is the Python runtime over it.
"""
from . import _lib  # noqa: F401
from ._lib import WvError, WV_FP32, WV_BF16, WV_FP8  # noqa: F401

__all__ = ["WvError", "WV_FP32", "WV_BF16", "WV_FP8"]
