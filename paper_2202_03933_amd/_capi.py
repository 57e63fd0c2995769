"""ctypes binding of the C ABI in include/mortar_mi355x.h (same names).

Argument marshalling only: every step of the mortar path runs in the HIP
library.  Importing this module on a machine without the built library
raises, so no caller can silently fall back to anything else.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libmortar_mi355x.so")

MT_OK, MT_EINVAL, MT_ECAPACITY, MT_EHIP, MT_ENOCONV, MT_EDEGENERATE, MT_ESTATE, MT_EUNSUPPORTED = range(8)
MT_SIDE_SLAVE, MT_SIDE_MASTER = 0, 1
MT_BASIS_STANDARD, MT_BASIS_DUAL = 0, 1
MT_NORMALS_ELEMENT, MT_NORMALS_NODAL = 0, 1

_NAMES = {0: "MT_OK", 1: "MT_EINVAL", 2: "MT_ECAPACITY", 3: "MT_EHIP", 4: "MT_ENOCONV", 5: "MT_EDEGENERATE",
          6: "MT_ESTATE", 7: "MT_EUNSUPPORTED"}


class mt_params(ctypes.Structure):
    _fields_ = [("delta", ctypes.c_double), ("bin_size", ctypes.c_double), ("lm_basis", ctypes.c_int32),
                ("rule", ctypes.c_int32), ("eps_d", ctypes.c_double), ("eps_a", ctypes.c_double),
                ("newton_tol", ctypes.c_double), ("newton_maxit", ctypes.c_int32), ("element_rule", ctypes.c_int32),
                ("normals", ctypes.c_int32), ("single_stream", ctypes.c_int32)]


class mt_stats(ctypes.Structure):
    _fields_ = [("n_candidates", ctypes.c_int64), ("n_pairs", ctypes.c_int64),
                ("nverts_hist", ctypes.c_int64 * 17), ("n_noconv", ctypes.c_int64),
                ("n_overflow", ctypes.c_int64), ("n_degenerate_slave", ctypes.c_int64),
                ("n_degenerate_master", ctypes.c_int64), ("n_lost_pairs", ctypes.c_int64),
                ("nnz_D", ctypes.c_int64), ("nnz_M", ctypes.c_int64),
                ("n_bins", ctypes.c_int64 * 3), ("bin_size", ctypes.c_double * 3)]


class mt_capacity(ctypes.Structure):
    _fields_ = [("candidates", ctypes.c_int64), ("screened", ctypes.c_int64), ("pairs", ctypes.c_int64),
                ("cells", ctypes.c_int64)]


MT_T_NAMES = ["prep", "bin_sort", "cand", "clip", "compact", "pattern", "pair_poly", "pair_fwd", "assemble",
              "pair_bwd", "grad_reduce"]
MT_T_COUNT = len(MT_T_NAMES)


class mt_timings(ctypes.Structure):
    _fields_ = [("ms", ctypes.c_double * MT_T_COUNT), ("intervals", ctypes.c_int64 * MT_T_COUNT)]


class mt_batch_tuning(ctypes.Structure):
    _fields_ = [("bucket", ctypes.c_int32), ("block", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


# name -> (restype, argtypes); every entry point of the header
_vp, _i32, _i64, _int = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_int
_pi64 = ctypes.POINTER(ctypes.c_int64)
_pi32 = ctypes.POINTER(ctypes.c_int32)
_psz = ctypes.POINTER(ctypes.c_size_t)
_pcap = ctypes.POINTER(mt_capacity)
SIGNATURES = {
    "mt_create": (_int, [ctypes.POINTER(_vp), _int]),
    "mt_destroy": (_int, [_vp]),
    "mt_default_params": (_int, [ctypes.POINTER(mt_params)]),
    "mt_set_params": (_int, [_vp, ctypes.POINTER(mt_params)]),
    "mt_upload": (_int, [_vp, _int, _i64, _vp, _vp, _vp, _i64, _vp, _vp]),
    "mt_update_coordinates": (_int, [_vp, _int, _vp, _vp, _vp, _vp]),
    "mt_default_capacity": (_int, [_vp, _pcap]),
    "mt_workspace_size": (_int, [_vp, _pcap, _psz]),
    "mt_build_pairs": (_int, [_vp, _pcap, _vp, ctypes.c_size_t, _pi64, _pi64, _vp]),
    "mt_build_pairs_static": (_int, [_vp, _pcap, _pi64, _pi64, _vp]),
    "mt_required_capacity": (_int, [_vp, _pcap]),
    "mt_check": (_int, [_vp]),
    "mt_get_pairs": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "mt_get_candidates": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "mt_csr_pattern": (_int, [_vp, _pi64, _pi64, _vp]),
    "mt_get_csr": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "mt_integrate": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "mt_backward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mt_integrate_backward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "mt_get_stats": (_int, [_vp, ctypes.POINTER(mt_stats)]),
    "mt_last_error": (ctypes.c_char_p, []),
    "mt_set_timing": (_int, [_vp, _int]),
    "mt_set_timing_phases": (_int, [_vp, ctypes.c_uint32]),
    "mt_get_timings": (_int, [_vp, ctypes.POINTER(mt_timings), _int]),
    "mt_batch_create": (_int, [ctypes.POINTER(_vp), _int]),
    "mt_batch_destroy": (_int, [_vp]),
    "mt_batch_add": (_int, [_vp, _vp, _pi32]),
    "mt_batch_workspace_size": (_int, [_vp, _psz]),
    "mt_batch_build": (_int, [_vp, ctypes.POINTER(mt_batch_tuning), _vp, ctypes.c_size_t, _vp]),
    "mt_batch_forward": (_int, [_vp, _vp, _vp, _vp, _int, _vp]),
    "mt_batch_backward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _int, _vp]),
    "mt_batch_search": (_int, [_vp, ctypes.c_int, _vp]),
    "mt_batch_autotune": (_int, [_vp, ctypes.POINTER(mt_batch_tuning), _vp]),
}

_lib = None


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build())")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


class MortarError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != MT_OK:
        raise MortarError(code, lib().mt_last_error().decode(errors="replace"))
    return code


def exported_symbols():
    return list(SIGNATURES)
