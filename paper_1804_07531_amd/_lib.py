"""ctypes declarations of the C ABI in include/rsvd.h.

Loading fails loudly when librsvd.so has not been built: there is no
fallback implementation of any step.
"""

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librsvd.so")

RSVD_OK, RSVD_EINVAL, RSVD_ESHAPE, RSVD_EWORKSPACE, RSVD_EBREAKDOWN, RSVD_EHIP, RSVD_EUNSUPPORTED = range(7)
RSVD_F64, RSVD_F32, RSVD_BF16, RSVD_FP8_E4M3 = range(4)
ALGO_SUBSPACE, ALGO_SINGLE_PASS, ALGO_BLOCK_KRYLOV = range(3)
KRYLOV_ALTERNATING, KRYLOV_ROW_SWEEP, KRYLOV_COL_SWEEP = range(3)
F32_MFMA, F32_BF16X6 = range(2)
ONE_VIEW_TROPP, ONE_VIEW_WOOLFE = range(2)
LC_FULL, LC_FIXED, LC_RATIO, LC_MINVAR = range(4)
CORE_GAUSSIAN, CORE_SRFT = range(2)
NORMAL_NYSTROM, NORMAL_PINCHED, NORMAL_SUBSPACE = range(3)
# bits of the device status word (rsvd_device_status)
FLAG_SHIFTED, FLAG_PIVOT, FLAG_NONFINITE, FLAG_TRUNCATED, FLAG_SYNC_TIMEOUT, FLAG_BAD_ENTRY = 1, 2, 4, 8, 16, 32

# exported symbols and their signatures (kept in the order of include/rsvd.h)
_c = ctypes


class RsvdMat(_c.Structure):
    _fields_ = [("dtype", _c.c_int), ("m", _c.c_int64), ("n", _c.c_int64), ("ld", _c.c_int64),
                ("trans", _c.c_int), ("data", _c.c_void_p), ("row_scale", _c.c_void_p)]


class RsvdViewTrace(_c.Structure):
    _fields_ = [("events", _c.POINTER(_c.c_void_p)), ("capacity", _c.c_int), ("used", _c.c_int),
                ("kind", _c.POINTER(_c.c_int)), ("inner", _c.c_int)]


class RsvdOpts(_c.Structure):
    _fields_ = [("seed", _c.c_uint64), ("refine", _c.c_int), ("krylov_mode", _c.c_int),
                ("block_rows", _c.c_int64), ("psi_rows", _c.c_int64), ("core_rows", _c.c_int),
                ("trunc_tau", _c.c_double), ("f32_mode", _c.c_int), ("trace", _c.POINTER(RsvdViewTrace)),
                ("one_view_method", _c.c_int), ("lc_rule", _c.c_int), ("lc", _c.c_int), ("lc_alpha", _c.c_double),
                ("core_kind", _c.c_int), ("sync_spins", _c.c_uint32)]


class RsvdBatchTuning(_c.Structure):
    _fields_ = [("plan_cus", _c.c_int), ("view_mr", _c.c_int)]


class RsvdOut(_c.Structure):
    _fields_ = [("U", _c.c_void_p), ("S", _c.c_void_p), ("V", _c.c_void_p)]


_P = _c.POINTER
SIGNATURES = {
    "rsvd_default_opts": (None, [_P(RsvdOpts)]),
    "rsvd_workspace_bytes": (_c.c_size_t, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts)]),
    "rsvd_subspace": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _P(RsvdOut),
                                 _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_subspace_noalloc": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _P(RsvdOut),
                                         _c.c_void_p]),
    "rsvd_noalloc_max_bytes": (_c.c_size_t, []),
    "rsvd_single_pass": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _P(RsvdOut),
                                    _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_block_krylov": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _P(RsvdOut),
                                     _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_device_status": (_c.c_int, [_c.c_void_p, _c.c_void_p, _P(_c.c_uint32)]),
    "rsvd_status_string": (_c.c_char_p, [_c.c_int]),
    "rsvd_one_view_lc": (_c.c_int, [_c.c_void_p, _c.c_void_p, _P(_c.c_int)]),
    "rsvd_extended_sizes": (_c.c_int, [_c.c_int, _c.c_int64, _c.c_int64, _c.c_int64, _P(_c.c_int),
                                       _P(_c.c_int64)]),
    "rsvd_gaussian": (_c.c_int, [_c.c_uint64, _c.c_uint32, _c.c_uint32, _c.c_int64, _c.c_int64, _c.c_int,
                                 _c.c_int, _c.c_void_p, _c.c_int64, _c.c_void_p]),
    "rsvd_view_range": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_void_p, _c.c_void_p, _P(RsvdOpts), _c.c_void_p,
                                   _c.c_size_t, _c.c_void_p]),
    "rsvd_view_corange": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_void_p, _c.c_void_p, _P(RsvdOpts), _c.c_void_p,
                                     _c.c_size_t, _c.c_void_p]),
    "rsvd_view_workspace_bytes": (_c.c_size_t, [_P(RsvdMat), _c.c_int, _P(RsvdOpts)]),
    "rsvd_philox_words": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_uint32, _c.c_uint32, _c.c_void_p,
                                     _c.c_void_p]),
    "rsvd_block_krylov_grad": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _P(RsvdOut),
                                          _c.c_void_p, _c.c_void_p, _c.c_double, _c.c_void_p, _c.c_int64,
                                          _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_grad_workspace_bytes": (_c.c_size_t, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts),
                                                _c.c_int]),
    "rsvd_block_krylov_grad_kept": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts),
                                               _P(RsvdOut), _c.c_void_p, _c.c_void_p, _c.c_double, _c.c_void_p,
                                               _c.c_int64, _c.c_void_p, _c.c_int, _c.c_void_p, _c.c_size_t,
                                               _c.c_void_p]),
    "rsvd_grad_kept_doubles": (_c.c_size_t, [_c.c_int, _c.c_int, _c.c_int]),
    "rsvd_default_batch_tuning": (None, [_P(RsvdBatchTuning)]),
    "rsvd_batch_plan_create": (_c.c_int, [_c.c_int, _P(RsvdMat), _P(_c.c_int), _c.c_int, _c.c_int, _P(RsvdOpts),
                                          _P(RsvdOut), _P(RsvdBatchTuning), _P(_c.c_void_p), _P(_c.c_size_t)]),
    "rsvd_batch_plan_bind": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_subspace_batched": (_c.c_int, [_c.c_void_p, _c.c_void_p]),
    "rsvd_batch_plan_launches": (_c.c_int, [_c.c_void_p]),
    "rsvd_batch_plan_destroy": (None, [_c.c_void_p]),
    "rsvd_normal_tevd": (_c.c_int, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts), _c.c_void_p,
                                    _c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_normal_workspace_bytes": (_c.c_size_t, [_P(RsvdMat), _c.c_int, _c.c_int, _c.c_int, _c.c_int,
                                                  _P(RsvdOpts)]),
    "rsvd_stream_create": (_c.c_int, [_c.c_int64, _c.c_int64, _c.c_int, _c.c_int, _c.c_int, _P(RsvdOpts),
                                      _P(_c.c_void_p), _P(_c.c_size_t)]),
    "rsvd_stream_bind": (_c.c_int, [_c.c_void_p, _c.c_void_p, _c.c_size_t, _c.c_void_p]),
    "rsvd_stream_add_dense": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_int64, _P(RsvdMat), _c.c_void_p]),
    "rsvd_stream_add_entries": (_c.c_int, [_c.c_void_p, _c.c_int64, _c.c_void_p, _c.c_void_p, _c.c_void_p,
                                           _c.c_void_p]),
    "rsvd_stream_finish": (_c.c_int, [_c.c_void_p, _P(RsvdOut), _c.c_void_p]),
    "rsvd_stream_destroy": (None, [_c.c_void_p]),
}

_lib = None


def load():
    """Load librsvd.so (once) and declare every exported function."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    lib = _c.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class RsvdError(RuntimeError):
    def __init__(self, code, where, flags=None):
        lib = load()
        msg = lib.rsvd_status_string(code).decode()
        extra = f", device flags {flags:#x}" if flags is not None else ""
        super().__init__(f"{where}: {msg} (status {code}{extra})")
        self.code = code
        self.flags = flags


def check(code, where):
    if code != RSVD_OK:
        raise RsvdError(code, where)
