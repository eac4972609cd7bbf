"""ctypes loader of libcvqkd_recon.so.  There is no fallback: if the library
is missing the import of the binding fails with instructions."""
from __future__ import annotations

import ctypes as C
from pathlib import Path

LIB_PATH = Path(__file__).resolve().parent / "libcvqkd_recon.so"

CVR_OK, CVR_EINVAL, CVR_ENOMEM, CVR_EHIP, CVR_EUNSUPPORTED = 0, -1, -2, -3, -4
STATUS_NAMES = {0: "CVR_OK", -1: "CVR_EINVAL", -2: "CVR_ENOMEM", -3: "CVR_EHIP", -4: "CVR_EUNSUPPORTED"}


class CvrError(RuntimeError):
    def __init__(self, status: int, fn: str, msg: str):
        super().__init__(f"{fn}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Frame(C.Structure):
    _fields_ = [("code_idx", C.c_int32), ("reserved", C.c_int32),
                ("vn_offset", C.c_int64), ("chk_offset", C.c_int64)]


class DecodeParams(C.Structure):
    _fields_ = [("algo", C.c_int32), ("max_iter", C.c_int32), ("early_stop", C.c_int32),
                ("math", C.c_int32), ("store", C.c_int32), ("alpha", C.c_float),
                ("msg_clamp", C.c_float), ("schedule", C.c_int32), ("wg_threads", C.c_int32), ("min_waves", C.c_int32), ("lds_cache_kb", C.c_int32), ("group_wgs", C.c_int32),
                ("weights", C.c_void_p),
                ("trace", C.c_void_p)]


# every extern "C" entry point and its signature
_P, _I32, _I64, _U32, _D = C.c_void_p, C.c_int32, C.c_int64, C.c_uint32, C.c_double
SIGNATURES = {
    "cvr_last_error": ([], C.c_char_p),
    "cvr_version": ([], C.c_int32),
    "cvr_code_create_csr": ([_I32, _I32, _P, _P, _P, _I32, _P], C.c_int),
    "cvr_code_create_qc": ([_I32, _I32, _I32, _P, _P, _I32, _P], C.c_int),
    "cvr_code_info": ([_P, _P, _P, _P, _P, _P], C.c_int),
    "cvr_code_destroy": ([_P], C.c_int),
    "slice_quantize": ([_P, _I64, _P, _I32, _I32, _P, _P], C.c_int),
    "slice_llr": ([_P, _I64, _D, _P, _I32, _I32, _I32, _U32, _P, _I32, _P, _P], C.c_int),
    "slice_llr_prior": ([_P, _I64, _D, _P, _I32, _I32, _I32, _U32, _P, _U32, _P, _I32, _P, _P], C.c_int),
    "slice_llr_bsc": ([_P, _I64, _P, _I32, _I32, _I32, _D, _I32, _P, _P], C.c_int),
    "slice_llr_next": ([_P, _I64, _D, _P, _I32, _I32, _I32, _U32, _P, _I32, _P, _P, _P, _P], C.c_int),
    "slice_llr_choose": ([_P, _P, _P, _I64, _I32, _P, _P], C.c_int),
    "syndrome_check": ([_P, _I32, _P, _P, _P, _P, _P], C.c_int),
    "cvr_batch_create": ([_P, _I32, _P, _I32, _P], C.c_int),
    "cvr_batch_info": ([_P, _P, _P, _P, _P], C.c_int),
    "cvr_batch_destroy": ([_P], C.c_int),
    "cvr_decode_workspace_size": ([_P, _P, _P], C.c_int),
    "ldpc_decode_batch": ([_P, _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P], C.c_int),
    "ldpc_decode_batch_noalloc": ([_P, _P, _P, _P, _P, _P, _P, _P, _P], C.c_int),
    "nms_unrolled_sizes": ([_P, _I32, _I32, _P, _P, _P], C.c_int),
    "nms_unrolled_fwd": ([_P, _I32, _I32, _P, _P, _P, _P, _P, _P, C.c_size_t, _P], C.c_int),
    "nms_unrolled_bwd": ([_P, _I32, _I32, _P, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P], C.c_int),
    "cvr_profile_enable": ([_I32], C.c_int),
    "cvr_profile_read": ([_I32, _P, _P, _I32], C.c_int),
    "cvr_debug_group_wait_ticks": ([C.c_uint64], C.c_int),
}

_lib = None


def load():
    """Loads the HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not LIB_PATH.exists():
            raise RuntimeError(
                f"{LIB_PATH} is missing: build it with `python -c 'import __graft_entry__ as g; g.build()'` "
                "(hipcc --offload-arch=gfx950).  There is no CPU fallback.")
        lib = C.CDLL(str(LIB_PATH))
        for name, (args, res) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def check(status: int, fn: str):
    if status != CVR_OK:
        raise CvrError(status, fn, load().cvr_last_error().decode(errors="replace"))
