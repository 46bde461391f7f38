"""ctypes declarations of the C ABI in include/rsr.h (argument marshalling only).

Every function keeps the C name.  Raw functions return the rsr_status code;
`check(ctx, status)` raises RSRError with the context's message.
"""
import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
# RSR_LIB names another build of the same library (for example one built with
# different kernel options); by default the in-tree build is loaded.
LIB_PATH = os.environ.get("RSR_LIB") or os.path.join(_HERE, "librsr.so")

RSR_OK, RSR_EINVAL, RSR_ENOMEM, RSR_EHIP, RSR_EUNSUPPORTED = 0, 1, 2, 3, 4
RSR_LABEL, RSR_COUNT = 0, 1
RSR_AUTO, RSR_POPCOUNT, RSR_MFMA, RSR_MFMA_FP4, RSR_PERSIST = 0, 1, 2, 3, 4
RSR_UNKNOWN_ONLY, RSR_ALL = 0, 1
RSR_SYS_ST_CONNECTIVITY = 1
RSR_SYS_GLOBAL_CONNECTIVITY = 2
RSR_SYS_MAX_FLOW = 3
RSR_SYS_HOST_CALLBACK = 4
RSR_MAX_K = 16
RSR_MAX_BITS = 4096
RSR_MAX_NODES = 4096


class rsr_estimate_t(ctypes.Structure):
    _fields_ = [("n_L", ctypes.c_uint64), ("n_U", ctypes.c_uint64), ("n_u", ctypes.c_uint64),
                ("n_both", ctypes.c_uint64), ("n_u_up", ctypes.c_uint64), ("N", ctypes.c_uint64),
                ("p_L", ctypes.c_double), ("p_U", ctypes.c_double), ("p_u", ctypes.c_double),
                ("P", ctypes.c_double), ("se", ctypes.c_double), ("cov", ctypes.c_double)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


# int32_t (*phi)(const uint8_t* x, int32_t n, void* user)
PHI_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.POINTER(ctypes.c_uint8), ctypes.c_int32,
                          ctypes.c_void_p)


class rsr_system_desc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("n_nodes", ctypes.c_int32),
                ("n_edges", ctypes.c_int32), ("K", ctypes.c_int32),
                ("edge_u", ctypes.POINTER(ctypes.c_int32)),
                ("edge_v", ctypes.POINTER(ctypes.c_int32)),
                ("source", ctypes.c_int32), ("sink", ctypes.c_int32), ("level", ctypes.c_int32),
                ("phi", PHI_FN), ("user", ctypes.c_void_p)]


class rsr_job(ctypes.Structure):
    _fields_ = [("model", ctypes.c_void_p), ("refs", ctypes.c_void_p), ("sys", ctypes.c_void_p),
                ("seed", ctypes.c_uint64), ("stream_id", ctypes.c_uint32), ("N", ctypes.c_int64),
                ("d_samples", ctypes.c_void_p), ("d_flags", ctypes.c_void_p),
                ("d_Y", ctypes.c_void_p), ("d_G", ctypes.c_void_p)]


class rsr_stage1_params(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int64), ("picks", ctypes.c_int64), ("eps_u", ctypes.c_double),
                ("max_rows", ctypes.c_int64), ("max_iters", ctypes.c_int32),
                ("seed", ctypes.c_uint64)]


class rsr_stage1_result(ctypes.Structure):
    _fields_ = [("iterations", ctypes.c_int32), ("p_u", ctypes.c_double), ("R_L", ctypes.c_int64),
                ("R_U", ctypes.c_int64), ("searches", ctypes.c_int64),
                ("duplicates", ctypes.c_int64)]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


_vp = ctypes.c_void_p
_pp = ctypes.POINTER(ctypes.c_void_p)
_i32, _i64, _u32, _u64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64

SIGNATURES = {
    "rsr_ctx_create": (ctypes.c_int, [ctypes.c_int, _vp, _pp]),
    "rsr_ctx_destroy": (ctypes.c_int, [_vp]),
    "rsr_last_error": (ctypes.c_char_p, [_vp]),
    "rsr_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "rsr_words": (ctypes.c_size_t, [_i32, _i32]),
    "rsr_thresholds": (ctypes.c_int, [_i32, _i32, _vp, _vp]),
    "rsr_model_create": (ctypes.c_int, [_vp, _i32, _i32, _vp, _pp]),
    "rsr_model_destroy": (ctypes.c_int, [_vp]),
    "rsr_model_update": (ctypes.c_int, [_vp, _vp]),
    "rsr_refs_create": (ctypes.c_int, [_vp, _i32, _i32, _vp, _i64, _vp, _i64, _pp]),
    "rsr_refs_destroy": (ctypes.c_int, [_vp]),
    "rsr_refs_consistent": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int32)]),
    "rsr_system_create": (ctypes.c_int, [_vp, ctypes.POINTER(rsr_system_desc), _pp]),
    "rsr_system_destroy": (ctypes.c_int, [_vp]),
    "rsr_sample": (ctypes.c_int, [_vp, _vp, _u64, _u32, _u64, _i64, _vp]),
    "rsr_classify": (ctypes.c_int, [_vp, _vp, _vp, _i64, _i32, _i32, _vp, _vp]),
    "rsr_eval_unknown": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp]),
    "rsr_eval_unknown_noalloc": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i32, _vp, _vp]),
    "rsr_estimate": (ctypes.c_int, [_vp, _vp, _vp, _i64, ctypes.POINTER(rsr_estimate_t)]),
    "rsr_grad": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp, _vp]),
    "rsr_importance": (ctypes.c_int, [_vp, _vp, _vp, _vp, _i64, _vp]),
    "rsr_boundary_search": (ctypes.c_int, [_vp, _vp, _vp, _i64, _vp, _i64, _vp, _vp]),
    "rsr_stage1": (ctypes.c_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp, _i64, _vp, _i64, _vp,
                                  _i64, _vp]),
    "rsr_plan_create": (ctypes.c_int, [_vp, ctypes.POINTER(rsr_job), _i32, ctypes.c_char_p, _pp]),
    "rsr_plan_run": (ctypes.c_int, [_vp]),
    "rsr_plan_results": (ctypes.c_int, [_vp, ctypes.POINTER(rsr_estimate_t), _vp]),
    "rsr_plan_destroy": (ctypes.c_int, [_vp]),
    "rsr_debug_fail_alloc": (ctypes.c_int, [_i64]),
    "rsr_debug_barrier_timeout": (ctypes.c_int, [_i64]),
}

_lib = None


class RSRError(RuntimeError):
    def __init__(self, status, message):
        self.status = status
        super().__init__(f"{_status_name(status)}: {message}")


def _status_name(s):
    return {0: "RSR_OK", 1: "RSR_EINVAL", 2: "RSR_ENOMEM", 3: "RSR_EHIP",
            4: "RSR_EUNSUPPORTED"}.get(s, f"status {s}")


def lib():
    """The loaded librsr.so.  Raises ImportError when the HIP library is not built:
    there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with paper_2604_17066_amd/build.py "
                          "(hipcc, gfx950); there is no CPU fallback")
    handle = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(handle, name)
        fn.restype = res
        fn.argtypes = args
    _lib = handle
    return handle


def check(ctx, status):
    if status != RSR_OK:
        msg = ""
        if ctx:
            raw = lib().rsr_last_error(ctx)
            msg = raw.decode() if raw else ""
        raise RSRError(status, msg)
