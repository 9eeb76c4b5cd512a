"""ctypes loader for libsorsvd.so: argument marshalling only, no arithmetic.

The library must have been built (``paper_1804_00462_amd.build.build()``);
a missing library is an error, never a silent fallback.
"""
import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsorsvd.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "sorsvd.h")

c_i32, c_i64, c_u64, c_sz, c_dbl = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_size_t, ctypes.c_double
c_vp = ctypes.c_void_p

SORSVD_F64, SORSVD_F32, SORSVD_BF16, SORSVD_DIAG, SORSVD_F16 = 0, 1, 2, 3, 4

STATUS = {0: "ok", -1: "invalid argument", -2: "workspace too small", -3: "HIP runtime error",
          -4: "Jacobi sweep cap reached", -5: "non-finite input", -6: "tolerance not met",
          -7: "unsupported by the library"}


class SorsvdError(RuntimeError):
    def __init__(self, status, where):
        super().__init__(f"{where}: {STATUS.get(status, 'unknown')} ({status})")
        self.status = status


class Opts(ctypes.Structure):
    _fields_ = [("l", c_i64), ("max_sweeps", c_i32), ("refine", c_i32), ("residual", c_i32),
                ("split", c_i32), ("tile", c_i32), ("pass_efficient", c_i32), ("col_exp", c_vp),
                ("literal", c_i32), ("out_f32", c_i32)]


class Problem(ctypes.Structure):
    _fields_ = [("A", c_vp), ("lda", c_i64), ("m", c_i64), ("n", c_i64), ("k", c_i32), ("l", c_i32),
                ("q", c_i32), ("reserved", c_i32), ("seed", c_u64), ("U", c_vp), ("ldu", c_i64),
                ("S", c_vp), ("V", c_vp), ("ldv", c_i64)]


class AutoInfo(ctypes.Structure):
    _fields_ = [("k_used", c_i32), ("q_used", c_i32), ("used_fallback", c_i32), ("runs", c_i32),
                ("err", c_dbl), ("k_pred", c_dbl * 4), ("flags", c_i32), ("reserved", c_i32),
                ("err_stored", c_dbl)]


class BoundsInfo(ctypes.Structure):
    _fields_ = [("omega2_norm", c_dbl), ("omega1_pinv_norm", c_dbl), ("th5_fro", c_dbl), ("th5_2", c_dbl),
                ("th7_fro", c_dbl), ("th7_2", c_dbl)]


class RpcaInfo(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("rank", c_i32), ("nnz_s", c_i64), ("xi", c_dbl), ("lam", c_dbl),
                ("norm2", c_dbl)]


class Info(ctypes.Structure):
    _fields_ = [("a_fro", c_dbl), ("err_fro", c_dbl), ("err_fro_explicit", c_dbl),
                ("sweeps", c_i32), ("flags", c_i32), ("a_noise_rel", c_dbl)]


_SIGS = {
    "sorsvd_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64, c_i32, c_i32, c_vp]),
    "sorsvd": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_i64, c_i32, c_u64,
                       c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_sz, c_vp, c_vp]),
    "sorsvd_read_info": (c_i32, [c_vp, c_vp, c_vp]),
    "sorsvd_predict_kq": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_u64, c_vp, c_dbl, c_vp, c_vp, c_vp,
                                  c_vp, c_sz, c_vp]),
    "sorsvd_bounds_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64]),
    "sorsvd_bounds": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_i64, c_i64, c_i32, c_u64, c_vp, c_i64, c_vp, c_vp,
                              c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_noalloc": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_i64, c_i32, c_u64,
                               c_vp, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_vp]),
    "sorsvd_pack_f16": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp]),
    "sorsvd_philox_normal": (c_i32, [c_u64, c_u64, c_u64, c_i64, c_i64, c_vp, c_vp]),
    "sorsvd_step_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64, c_i32]),
    "sorsvd_step_sketch": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_step_orbit": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_step_qr": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_step_project": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_vp, c_vp, c_i64, c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_step_core_svd": (c_i32, [c_vp, c_i64, c_i64, c_vp, c_vp, c_vp, c_i32, c_vp, c_sz, c_vp]),
    "sorsvd_pass_timing": (c_i32, [c_i32, c_i32]),
    "sorsvd_pass_timing_read": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "sorsvd_batch_create": (c_i32, [c_i32, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "sorsvd_batch_upload": (c_i32, [c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_batch_run": (c_i32, [c_vp, c_vp, c_vp]),
    "sorsvd_batch_get_config": (c_i32, [c_vp, c_vp]),
    "sorsvd_batch_set_config": (c_i32, [c_vp, c_vp]),
    "sorsvd_batch_autotune": (c_i32, [c_vp, c_vp, c_vp, c_vp]),
    "sorsvd_batch_read_info": (c_i32, [c_vp, c_vp, c_vp]),
    "sorsvd_batch_graph": (c_i32, [c_vp, c_vp, c_vp]),
    "sorsvd_graph_launch": (c_i32, [c_vp, c_vp]),
    "sorsvd_graph_destroy": (c_i32, [c_vp]),
    "sorsvd_batch_count": (c_i32, [c_vp]),
    "sorsvd_batch_destroy": (None, [c_vp]),
    "sorsvd_probe_workspace_bytes": (c_sz, [c_i64, c_i64, c_i32]),
    "sorsvd_probe_features": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_u64, c_vp, c_vp, c_sz, c_vp]),
    "sorsvd_mlp_param_count": (c_i32, []),
    "sorsvd_mlp_work_floats": (c_sz, [c_i32]),
    "sorsvd_mlp_forward": (c_i32, [c_vp, c_vp, c_i32, c_vp, c_vp, c_vp]),
    "sorsvd_mlp_backward": (c_i32, [c_vp, c_vp, c_vp, c_i32, c_vp, c_vp, c_vp, c_vp]),
    "sorsvd_mlp_adam": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_i64, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                                ctypes.c_float, c_vp]),
    "sorsvd_mlp_train_step": (c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i32, c_i64, ctypes.c_float, c_vp, c_vp,
                                      c_vp, c_vp]),
    "sorsvd_rpca_workspace_bytes": (c_sz, [c_i64, c_i64, c_i64, c_i32]),
    "sorsvd_rpca": (c_i32, [c_vp, c_i64, c_i64, c_i64, c_i64, c_i32, c_u64, c_dbl, c_i32, c_vp, c_vp, c_i64,
                            c_vp, c_sz, c_vp, c_vp]),
    "sorsvd_auto_workspace_bytes": (c_sz, [c_i64, c_i64, c_i32]),
    "sorsvd_auto": (c_i32, [c_vp, c_i64, c_i32, c_i64, c_i64, c_u64, c_dbl, c_vp, c_vp, c_i64, c_vp, c_vp, c_i64,
                            c_vp, c_sz, c_vp, c_vp]),
    "sorsvd_status_string": (ctypes.c_char_p, [c_i32]),
    "sorsvd_version": (ctypes.c_char_p, []),
}

_lib = None


def header_symbols():
    """Function names declared in include/sorsvd.h."""
    with open(HEADER) as f:
        text = f.read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(sorsvd\w*)\s*\(", text)))


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1804_00462_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status, where):
    if status != 0:
        raise SorsvdError(status, where)
