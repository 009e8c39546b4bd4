"""ctypes binding of libwv.so (include/wv.h).  Argument marshalling only.

torch is imported first so that libwv.so binds to the HIP runtime torch has
already loaded (same SONAME): device pointers and streams are shared.
The library is loaded lazily and never built here; a missing library raises.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime before libwv.so)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libwv.so")

WV_OK, WV_EINVAL, WV_ESHAPE, WV_EORDER, WV_EDEVICE, WV_ECORRUPT, WV_EUNSUPPORTED, WV_ENOMEM = \
    0, -1, -2, -3, -4, -5, -6, -7
WV_FP32, WV_BF16, WV_FP8 = 0, 1, 2
WV_DIST_GAUSS, WV_DIST_LAPLACE = 0, 1
DISTS = {"gauss": WV_DIST_GAUSS, "laplace": WV_DIST_LAPLACE}
ERR_NAMES = {0: "WV_OK", -1: "WV_EINVAL", -2: "WV_ESHAPE", -3: "WV_EORDER", -4: "WV_EDEVICE",
             -5: "WV_ECORRUPT", -6: "WV_EUNSUPPORTED", -7: "WV_ENOMEM"}


class WvError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERR_NAMES.get(code, code)}: {msg}")
        self.code = code


class wv_config(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int), ("lift_ch", ctypes.c_int), ("lift_layers", ctypes.c_int),
                ("ctx_ch", ctypes.c_int), ("ctx_layers", ctypes.c_int), ("mix_k", ctypes.c_int),
                ("sym_min", ctypes.c_int), ("sym_max", ctypes.c_int), ("cdf_bits", ctypes.c_int),
                ("sigma_min", ctypes.c_float), ("lift_int", ctypes.c_int), ("dist", ctypes.c_int),
                ("ctx_arch", ctypes.c_int), ("ll_ar", ctypes.c_int), ("ar_ch", ctypes.c_int)]


class wv_group(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("nplanes", ctypes.c_int),
                ("d_q", ctypes.c_void_p), ("d_state", ctypes.c_void_p), ("d_scratch", ctypes.c_void_p)]


class wv_step_item(ctypes.Structure):
    _fields_ = [("H", ctypes.c_int), ("W", ctypes.c_int), ("nplanes", ctypes.c_int),
                ("d_q", ctypes.c_void_p), ("d_state", ctypes.c_void_p), ("d_scratch", ctypes.c_void_p),
                ("subband", ctypes.c_int), ("step", ctypes.c_int), ("d_params", ctypes.c_void_p)]


class wv_subband(ctypes.Structure):
    _fields_ = [("h", ctypes.c_int), ("w", ctypes.c_int), ("level", ctypes.c_int),
                ("type", ctypes.c_int), ("offset", ctypes.c_longlong)]


_P = ctypes.c_void_p
_I = ctypes.c_int
_LL = ctypes.c_longlong
_F = ctypes.c_float
_SZ = ctypes.c_size_t
_CFG = ctypes.POINTER(wv_config)

_SIGS = {
    "wv_last_error": (ctypes.c_char_p, []),
    "wv_version": (_I, []),
    "wv_weights_count": (_I, [_CFG, ctypes.POINTER(_LL)]),
    "wv_pack_bytes": (_I, [_CFG, _I, ctypes.POINTER(_SZ)]),
    "wv_model_create": (_I, [_CFG, _P, _LL, _I, _P, _SZ, _P, ctypes.POINTER(_P)]),
    "wv_model_destroy": (None, [_P]),
    "wv_layout": (_I, [_CFG, _I, _I, ctypes.POINTER(wv_subband), _I, ctypes.POINTER(_LL)]),
    "wv_group_count": (_LL, [_I, _I, _I]),
    "wv_workspace_bytes": (_I, [_P, _I, _I, _I, ctypes.POINTER(_SZ), ctypes.POINTER(_SZ)]),
    "wv_analyze": (_I, [_P, _P, _P, _I, _I, _I, _F, _F, _P, _P, _P, _P, _P]),
    "wv_context_params": (_I, [_P, _P, _I, _I, _I, _I, _I, _P, _P, _P, _P]),
    "wv_cdf_tables": (_I, [_P, _LL, _I, _I, _I, _I, _I, _P, _P]),
    "wv_ar_params": (_I, [_P, _P, _I, _I, _I, _P, _P]),
    "wv_ar_decode": (_I, [_P, _P, _P, _I, _I, _I, _P, _P, _P]),
    "wv_plan_bytes": (_I, [_P, _I, _P, _P, ctypes.POINTER(_SZ), ctypes.POINTER(_LL)]),
    "wv_plan_create": (_I, [_P, _I, _P, _P, _P, _SZ, _P, _P, ctypes.POINTER(_P)]),
    "wv_plan_destroy": (None, [_P]),
    "wv_plan_rows": (_I, [_P, _I, _I, ctypes.POINTER(_LL), _P]),
    "wv_plan_context_params": (_I, [_P, _I, _I, _P]),
    "wv_plan_scatter": (_I, [_P, _P, _I, _I, _P]),
    "wv_context_params_items": (_I, [_P, _I, _P, _P, _SZ, _P, _SZ, ctypes.POINTER(_SZ), _P]),
    "wv_scatter_symbols": (_I, [_CFG, _P, _I, _I, _I, _I, _I, _P, _P]),
    "wv_gather_symbols": (_I, [_CFG, _P, _I, _I, _I, _I, _I, _P, _P]),
    "wv_synthesize": (_I, [_P, _P, _P, _I, _I, _I, _F, _F, _F, _P, _P, _P, _P]),
    "wv_center_u8": (_I, [_P, _LL, _P, _P]),
    "wv_add_offset": (_I, [_P, _LL, _F, _P, _P]),
    "wv_impulse_scratch_bytes": (_I, [_P, ctypes.POINTER(_SZ)]),
    "wv_impulse_responses": (_I, [_P, _P, _I, _I, _F, _F, _P, _P, _P]),
    "wv_temporal_haar_forward": (_I, [_P, _I, _LL, _P]),
    "wv_temporal_haar_inverse": (_I, [_P, _I, _LL, _P]),
    "wv_rans_encode": (_I, [_P, _I, _P, _LL, _P, _SZ, ctypes.POINTER(_SZ)]),
    "wv_rans_decode": (_I, [_P, _I, _LL, _P, _SZ, _P]),
    "wv_cdf_trim_scratch_bytes": (_I, [_LL, ctypes.POINTER(_SZ)]),
    "wv_cdf_trim": (_I, [_P, _LL, _I, _P, _P, _LL, _P, _SZ, _P]),
    "wv_cdf_trim_noalloc": (_I, [_P, _LL, _I, _P, _P, _LL, _P]),
    "wv_cdf_untrim": (_I, [_P, _P, _LL, _I, _LL, _P]),
    "wv_rans_encode_trim": (_I, [_P, _P, _LL, _I, _P, _LL, _P, _SZ, ctypes.POINTER(_SZ)]),
    "wv_rans_decode_trim": (_I, [_P, _P, _LL, _I, _LL, _P, _SZ, _P]),
    "wv_zero": (_I, [_P, _SZ, _P]),
    "wv_graph_begin": (_I, [_P]),
    "wv_graph_end": (_I, [_P, ctypes.POINTER(_P)]),
    "wv_graph_launch": (_I, [_P, _P]),
    "wv_graph_destroy": (None, [_P]),
}

_lib = None


def lib():
    """The loaded libwv.so; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2405_12631_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGS.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(rc):
    if rc != WV_OK:
        raise WvError(rc, lib().wv_last_error().decode(errors="replace"))
    return rc


def call(name, *args):
    """Call a wv_* function that returns a status code; raise WvError on failure."""
    return check(getattr(lib(), name)(*args))


def symbols():
    """Names of the exported entry points the binding knows."""
    return list(_SIGS)
