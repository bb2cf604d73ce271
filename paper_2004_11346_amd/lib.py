"""ctypes binding of ``libsht.so`` (the C-ABI in ``include/sht.h``).

Argument marshalling only.  The library is loaded from the package directory;
if it is missing this module raises -- there is no fallback implementation.
``torch`` is imported first so that the library binds to the same HIP runtime
as torch (both are ``libamdhip64.so.7``).
"""
from __future__ import annotations

import ctypes
import os
import threading

import torch  # noqa: F401  (must be loaded before libsht.so, see module doc)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsht.so")

SHT_OK = 0
SHT_F64, SHT_F32 = 0, 1
SHT_DENSE, SHT_IDBF = 0, 1
SHT_FWD, SHT_INV, SHT_ADJ = 0, 1, 2
SHT_F32_VALU, SHT_F32_SPLIT_BF16, SHT_F32_SPLIT_BF16_6 = 0, 1, 2
SHT_SAMPLE_MOCK_CHEB, SHT_SAMPLE_RANDOM = 0, 1
SHT_DFT_AUTO, SHT_DFT_ROWS, SHT_DFT_RADER, SHT_DFT_FOUR_STEP = 0, 1, 2, 3
SHT_LEVELS_AUTO, SHT_LEVELS_STAGED, SHT_LEVELS_FUSED = 0, 1, 2
SHT_ERR_INVALID_ARG, SHT_ERR_UNSUPPORTED, SHT_ERR_PLAN_CORRUPT = -1, -2, -7
SHT_GROUP_PERSISTENT, SHT_GROUP_BATCHED = 0, 1

EXPORTED = [
    "sht_plan_opts_default", "sht_plan_create", "sht_plan_destroy", "sht_forward", "sht_inverse",
    "sht_backward", "sht_alt_apply", "sht_plan_stats", "sht_profile", "sht_profile_report", "sht_plan_info", "sht_plan_nodes",
    "sht_strerror", "sht_last_error_detail", "sht_host_plan_create", "sht_host_plan_destroy",
    "sht_host_plan_apply", "sht_host_alt_matrix", "sht_host_plan_stats", "sht_host_gauss_legendre",
    "sht_group_create", "sht_group_destroy", "sht_group_bind", "sht_group_forward", "sht_group_inverse",
    "sht_group_tune", "sht_group_capture", "sht_group_replay", "sht_group_stats", "sht_inverse_noalloc",
    "sht_set_graph_capture", "sht_plan_cache_verify", "sht_plan_cache_path",
    "sht_forward_real", "sht_inverse_real", "sht_group_opts_default", "sht_group_create_ex",
    "sht_host_dft_tables",
]


class ShtError(RuntimeError):
    def __init__(self, code: int, what: str, detail: str):
        super().__init__(f"{what}: {detail or 'error'} (code {code})")
        self.code = code


class PlanOpts(ctypes.Structure):
    _fields_ = [
        ("eps", ctypes.c_double),
        ("n0", ctypes.c_int),
        ("leaf", ctypes.c_int),
        ("rk", ctypes.c_int),
        ("oversample", ctypes.c_int),
        ("rsvd_r", ctypes.c_int),
        ("rsvd_q", ctypes.c_int),
        ("sampling", ctypes.c_int),
        ("seed", ctypes.c_uint64),
        ("threads", ctypes.c_int),
        ("f32_mode", ctypes.c_int),
        ("min_idbf", ctypes.c_int),
        ("dense_gen", ctypes.c_int),
        ("m_lo", ctypes.c_int),
        ("m_hi", ctypes.c_int),
        ("dft_schedule", ctypes.c_int),
        ("id_check", ctypes.c_int),
        ("cache_dir", ctypes.c_char_p),
        ("level_schedule", ctypes.c_int),
    ]


class GroupOpts(ctypes.Structure):
    _fields_ = [("mode", ctypes.c_int), ("tune_file", ctypes.c_char_p), ("plan_cache_dir", ctypes.c_char_p)]


_lock = threading.Lock()
_lib = None


def load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"native library {LIB_PATH} is missing; build it with "
                "`python -m paper_2004_11346_amd.build` (there is no non-native fallback)")
        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        I = ctypes.c_int
        PP = ctypes.POINTER(ctypes.c_void_p)
        lib.sht_plan_opts_default.argtypes = [ctypes.POINTER(PlanOpts)]
        lib.sht_plan_opts_default.restype = None
        lib.sht_plan_create.argtypes = [I, I, I, I, ctypes.POINTER(PlanOpts), PP]
        lib.sht_plan_destroy.argtypes = [P]
        lib.sht_plan_destroy.restype = None
        for n in ("sht_forward", "sht_inverse", "sht_backward", "sht_inverse_noalloc"):
            getattr(lib, n).argtypes = [P, P, P, P]
        lib.sht_alt_apply.argtypes = [P, I, I, I, P, P, P]
        lib.sht_set_graph_capture.argtypes = [P, I]
        lib.sht_forward_real.argtypes = [P, I, P, P, P]
        lib.sht_inverse_real.argtypes = [P, I, P, P, P]
        lib.sht_plan_cache_verify.argtypes = [ctypes.c_char_p]
        lib.sht_plan_cache_path.argtypes = [I, ctypes.POINTER(PlanOpts), ctypes.c_char_p, ctypes.c_size_t]
        lib.sht_plan_stats.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        lib.sht_profile.argtypes = [P, I]
        lib.sht_profile_report.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        lib.sht_plan_info.argtypes = [P, ctypes.POINTER(I), ctypes.POINTER(I), ctypes.POINTER(I),
                                      ctypes.POINTER(I)]
        lib.sht_plan_nodes.argtypes = [P, P, P]
        lib.sht_strerror.argtypes = [I]
        lib.sht_strerror.restype = ctypes.c_char_p
        lib.sht_last_error_detail.argtypes = []
        lib.sht_last_error_detail.restype = ctypes.c_char_p
        lib.sht_host_plan_create.argtypes = [I, I, ctypes.POINTER(PlanOpts), PP]
        lib.sht_host_plan_destroy.argtypes = [P]
        lib.sht_host_plan_destroy.restype = None
        lib.sht_host_plan_apply.argtypes = [P, I, I, I, I, P, P]
        lib.sht_host_alt_matrix.argtypes = [P, I, I, P]
        lib.sht_host_plan_stats.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        lib.sht_host_gauss_legendre.argtypes = [I, P, P]
        lib.sht_host_dft_tables.argtypes = [I, I, I, ctypes.c_char_p, ctypes.c_size_t]
        lib.sht_group_create.argtypes = [I, P, P, I, PP]
        lib.sht_group_opts_default.argtypes = [ctypes.POINTER(GroupOpts)]
        lib.sht_group_opts_default.restype = None
        lib.sht_group_create_ex.argtypes = [I, P, P, I, ctypes.POINTER(GroupOpts), PP]
        lib.sht_group_destroy.argtypes = [P]
        lib.sht_group_destroy.restype = None
        lib.sht_group_bind.argtypes = [P, P, P]
        for n in ("sht_group_forward", "sht_group_inverse", "sht_group_tune"):
            getattr(lib, n).argtypes = [P, P]
        lib.sht_group_capture.argtypes = [P, I, P]
        lib.sht_group_replay.argtypes = [P, I, P]
        lib.sht_group_stats.argtypes = [P, ctypes.c_char_p, ctypes.c_size_t]
        for n in EXPORTED:
            f = getattr(lib, n)
            if f.restype is ctypes.c_int or n in ("sht_plan_create", "sht_forward", "sht_inverse",
                                                   "sht_backward", "sht_alt_apply", "sht_plan_stats",
                                                   "sht_plan_info", "sht_plan_nodes",
                                                   "sht_host_plan_create", "sht_host_plan_apply",
                                                   "sht_host_alt_matrix", "sht_host_plan_stats",
                                                   "sht_host_gauss_legendre", "sht_host_dft_tables"):
                f.restype = ctypes.c_int
        _lib = lib
        return lib


def check(rc: int, what: str):
    if rc < 0:
        lib = load()
        detail = lib.sht_last_error_detail().decode(errors="replace")
        msg = lib.sht_strerror(rc).decode()
        raise ShtError(rc, what, f"{msg}; {detail}")
    return rc


def default_opts(**kw) -> PlanOpts:
    o = PlanOpts()
    load().sht_plan_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        if not hasattr(o, k):
            raise TypeError(f"unknown plan option {k}")
        if k == "cache_dir" and isinstance(v, str):
            v = v.encode()
        setattr(o, k, v)
    return o
