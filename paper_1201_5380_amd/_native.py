"""ctypes loader for libdedisp.so (the gfx950 library built in-tree).

There is no fallback: if the library is missing or fails to load, every call
raises.  Argument marshalling only; all computation happens in the library.
"""
from __future__ import annotations

import ctypes
import os

PKG = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(PKG, "libdedisp.so")

OK = 0
STATUS_NAMES = {
    0: "DEDISP_OK", -1: "DEDISP_ERR_INVALID_ARG", -2: "DEDISP_ERR_NO_DM_LIST",
    -3: "DEDISP_ERR_TOO_FEW_SAMPLES", -4: "DEDISP_ERR_OOM", -5: "DEDISP_ERR_HIP",
    -6: "DEDISP_ERR_UNSUPPORTED",
}

# Every entry point declared in include/dedisp.h, with (restype, argtypes).
_vp = ctypes.c_void_p
_i = ctypes.c_int
_d = ctypes.c_double
_sz = ctypes.c_size_t
_u64 = ctypes.c_uint64
_pi = ctypes.POINTER(ctypes.c_int)
_psz = ctypes.POINTER(ctypes.c_size_t)
_pu64 = ctypes.POINTER(ctypes.c_uint64)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_pf64 = ctypes.POINTER(ctypes.c_double)
_pf32 = ctypes.POINTER(ctypes.c_float)


class TileConfig(ctypes.Structure):
    _fields_ = [("kind", _i), ("waves", _i), ("dms_per_wave", _i),
                ("words_per_lane", _i), ("chunk_chans", _i), ("sample_format", _i)]

    def as_dict(self):
        return {f: getattr(self, f) for f, _ in self._fields_}


class BeamStruct(ctypes.Structure):
    _fields_ = [("plan", _vp), ("d_in", _vp), ("nsamps", _sz), ("d_out", _vp),
                ("out_row_stride", _sz)]


_PTC = ctypes.POINTER(TileConfig)

SIGNATURES = {
    "dedisp_status_string": (ctypes.c_char_p, [_i]),
    "dedisp_last_error": (ctypes.c_char_p, []),
    "dedisp_plan_create": (_i, [ctypes.POINTER(_vp), _i, _d, _d, _d, _i]),
    "dedisp_plan_destroy": (None, [_vp]),
    "dedisp_set_dm_list": (_i, [_vp, _pf64, _i]),
    "dedisp_set_killmask": (_i, [_vp, _pi32]),
    "dedisp_get_nchans": (_i, [_vp, _pi]),
    "dedisp_get_nbits": (_i, [_vp, _pi]),
    "dedisp_get_dm_count": (_i, [_vp, _pi]),
    "dedisp_get_max_delay": (_i, [_vp, _pi]),
    "dedisp_get_delay_table": (_i, [_vp, _pi32]),
    "dedisp_execute": (_i, [_vp, _vp, _sz, _vp, _sz, _vp]),
    "dedisp_execute_noalloc": (_i, [_vp, _vp, _sz, _vp, _sz, _vp]),
    "dedisp_get_diagonal_dm": (_i, [_vp, ctypes.POINTER(_d)]),
    "dedisp_default_scrunch_factors": (_i, [_vp, _i, _pi32]),
    "dedisp_set_scrunching": (_i, [_vp, _pi32]),
    "dedisp_get_output_lengths": (_i, [_vp, _sz, _psz]),
    "dedisp_set_subband": (_i, [_vp, _i, _i]),
    "dedisp_set_tree": (_i, [_vp, _i]),
    "dedisp_set_output_format": (_i, [_vp, _i, _i]),
    "dedisp_get_output_format": (_i, [_vp, _pi, _pi]),
    "dedisp_tile_config_count": (_i, []),
    "dedisp_tile_config_get": (_i, [_i, _PTC]),
    "dedisp_set_tile_config": (_i, [_vp, _PTC]),
    "dedisp_get_tile_config": (_i, [_vp, _PTC]),
    "dedisp_tune": (_i, [_vp, _vp, _sz, _vp, _sz, _vp, ctypes.c_char_p, _pf32]),
    "dedisp_stream_create": (_i, [_vp, ctypes.POINTER(_vp)]),
    "dedisp_stream_destroy": (None, [_vp]),
    "dedisp_stream_push": (_i, [_vp, _vp, _sz, _vp, _sz, _psz, _vp]),
    "dedisp_stream_reserve": (_i, [_vp, _sz]),
    "dedisp_stream_push_many": (_i, [ctypes.POINTER(_vp), ctypes.POINTER(_vp), _psz,
                                     ctypes.POINTER(_vp), _psz, _psz, _i, _vp]),
    "dedisp_stream_get_state": (_i, [_vp, _psz, _pu64]),
    "dedisp_stream_get_device_bytes": (_i, [_vp, _psz]),
    "dedisp_stream_get_history": (_i, [_vp, _vp, _psz]),
    "dedisp_stream_set_history": (_i, [_vp, _vp, _sz, _u64]),
    "dedisp_stream_reset": (_i, [_vp]),
    "dedisp_batch_create": (_i, [ctypes.POINTER(BeamStruct), _i, ctypes.c_char_p, _vp,
                                 ctypes.POINTER(_vp)]),
    "dedisp_batch_execute": (_i, [_vp, _vp]),
    "dedisp_batch_execute_direct": (_i, [_vp, _vp]),
    "dedisp_batch_destroy": (None, [_vp]),
}

_lib = None


class DedispError(RuntimeError):
    def __init__(self, status, where):
        self.status = status
        msg = ""
        if _lib is not None:
            raw = _lib.dedisp_last_error()
            msg = raw.decode() if raw else ""
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}"
                         + (f" ({msg})" if msg else ""))


def lib():
    """The loaded library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_1201_5380_amd.build` "
            "(there is no fallback implementation)")
    # The library must share torch's HIP runtime (torch's device allocations
    # and streams are what it is handed).  torch bundles its own
    # libamdhip64.so (soname libamdhip64.so.7); loading torch first makes the
    # dynamic linker bind our NEEDED libamdhip64.so.7 to that same copy
    # instead of a second runtime from /opt/rocm.
    import torch  # noqa: F401
    handle = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    _lib = handle
    return handle


def check(status, where):
    if status != OK:
        raise DedispError(status, where)
    return status
