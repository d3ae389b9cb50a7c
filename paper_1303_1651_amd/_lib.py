"""ctypes binding of libspgemm.so (the C ABI in include/spgemm.h).

Argument marshalling only: every step of the product runs in the HIP
library.  Importing this module fails loudly when the library has not been
built; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspgemm.so")

if not os.path.exists(LIB_PATH):
    raise ImportError("libspgemm.so is not built: run `python -m paper_1303_1651_amd.build` "
                      "(or __graft_entry__.build()) first")

lib = ctypes.CDLL(LIB_PATH)

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32
SZ = ctypes.c_size_t
F32 = ctypes.c_float

SPGEMM_OK = 0
STATUS = {
    0: "SPGEMM_OK", 1: "SPGEMM_E_NULL", 2: "SPGEMM_E_DIM", 3: "SPGEMM_E_NOT_CANONICAL",
    4: "SPGEMM_E_INDEX_OVERFLOW", 5: "SPGEMM_E_WORKSPACE", 6: "SPGEMM_E_CAPACITY",
    7: "SPGEMM_E_NO_MODEL", 8: "SPGEMM_E_STATE", 9: "SPGEMM_E_HIP", 10: "SPGEMM_E_INVALID",
    11: "SPGEMM_E_IO",
}
SIZER_EXACT, SIZER_UPPER_BOUND, SIZER_LEARNED = 0, 1, 2
OPT_FAST, OPT_VALIDATE, OPT_TIMING = 1, 2, 4
MLP_PARAMS = 1217


class spgemm_csr(ctypes.Structure):
    _fields_ = [("rows", I64), ("cols", I64), ("nnz", I64),
                ("row_ptr", P), ("col_idx", P), ("val", P)]


class spgemm_tuning(ctypes.Structure):
    _fields_ = [("table_slots", I32), ("stage_slots", I32),
                ("merge_max_nnz", I32), ("merge_lists", I32), ("dense_ratio", F32),
                ("margin", F32), ("slack", I32), ("blocks_per_cu", I32),
                ("spill_ratio", F32), ("bitmap_cols", I32), ("split_merge", I32)]


class spgemm_options(ctypes.Structure):
    _fields_ = [("sizer", I32), ("flags", I32), ("model", P), ("tuning", ctypes.POINTER(spgemm_tuning))]


class spgemm_info(ctypes.Structure):
    _fields_ = [("multiplications", I64), ("c_capacity_hint", I64), ("c_nnz", I64),
                ("scratch_bytes", SZ), ("rows_merge", I64), ("rows_hash", I64),
                ("rows_global", I64), ("rows_empty", I64), ("overflow_rows", I64), ("spilled_rows", I64),
                ("tiles", I64),
                ("tile_ms", ctypes.c_double), ("tile_ms_total", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class spgemm_train_params(ctypes.Structure):
    _fields_ = [("epochs", I32), ("batch_size", I32), ("lr", F32), ("beta1", F32),
                ("beta2", F32), ("eps", F32)]


def _sig(name, restype, argtypes):
    f = getattr(lib, name)
    f.restype = restype
    f.argtypes = argtypes
    return f


CSR_P = ctypes.POINTER(spgemm_csr)
OPT_P = ctypes.POINTER(spgemm_options)
INFO_P = ctypes.POINTER(spgemm_info)
I64_P = ctypes.POINTER(I64)
SZ_P = ctypes.POINTER(SZ)
F32_P = ctypes.POINTER(F32)

spgemm_status_string = _sig("spgemm_status_string", ctypes.c_char_p, [ctypes.c_int])
spgemm_plan_workspace_size = _sig("spgemm_plan_workspace_size", ctypes.c_int, [CSR_P, CSR_P, OPT_P, SZ_P])
spgemm_plan_create = _sig("spgemm_plan_create", ctypes.c_int,
                          [CSR_P, CSR_P, OPT_P, P, SZ, P, ctypes.POINTER(P), INFO_P])
spgemm_symbolic = _sig("spgemm_symbolic", ctypes.c_int, [P, P, SZ, P, I64_P, P])
spgemm_numeric = _sig("spgemm_numeric", ctypes.c_int, [P, P, SZ, P, P, P, P, P, I64, I64_P, P])
spgemm_numeric_static = _sig("spgemm_numeric_static", ctypes.c_int, [P, P, P, P, P, P, I64, I64_P, P])
spgemm_numeric_static_limit = _sig("spgemm_numeric_static_limit", SZ, [])
spgemm_compute_only = _sig("spgemm_compute_only", ctypes.c_int, [P, P, P, P, P, P])
spgemm_plan_info = _sig("spgemm_plan_info", ctypes.c_int, [P, INFO_P])
spgemm_plan_last_hip_error = _sig("spgemm_plan_last_hip_error", ctypes.c_int, [P])
spgemm_plan_destroy = _sig("spgemm_plan_destroy", None, [P])

spgemm_model_create = _sig("spgemm_model_create", ctypes.c_int, [F32_P, F32_P, F32_P, ctypes.POINTER(P)])
spgemm_model_get = _sig("spgemm_model_get", ctypes.c_int, [P, F32_P, F32_P, F32_P])
spgemm_model_save = _sig("spgemm_model_save", ctypes.c_int, [P, ctypes.c_char_p])
spgemm_model_load = _sig("spgemm_model_load", ctypes.c_int, [ctypes.c_char_p, ctypes.POINTER(P)])
spgemm_model_destroy = _sig("spgemm_model_destroy", None, [P])
spgemm_model_device_bytes = _sig("spgemm_model_device_bytes", SZ, [])
spgemm_model_upload = _sig("spgemm_model_upload", ctypes.c_int, [P, P, P])
spgemm_row_features = _sig("spgemm_row_features", ctypes.c_int, [CSR_P, CSR_P, P, P, P, P])
spgemm_model_stats_scratch = _sig("spgemm_model_stats_scratch", SZ, [I64])
spgemm_model_feature_stats = _sig("spgemm_model_feature_stats", ctypes.c_int,
                                  [P, P, P, I64, F32_P, F32_P, P, P])
spgemm_model_grad_scratch = _sig("spgemm_model_grad_scratch", SZ, [I64])
spgemm_model_loss_grad = _sig("spgemm_model_loss_grad", ctypes.c_int,
                              [P, P, P, P, P, I64, P, P, F32_P, P])
spgemm_model_train_scratch = _sig("spgemm_model_train_scratch", SZ, [I64, I32])
spgemm_model_train = _sig("spgemm_model_train", ctypes.c_int,
                          [F32_P, F32_P, F32_P, P, P, P, P, I64, ctypes.POINTER(spgemm_train_params),
                           P, SZ, F32_P, ctypes.POINTER(P), P])
spgemm_model_predict = _sig("spgemm_model_predict", ctypes.c_int, [P, P, P, P, I64, P, P, P])

EXPORTED = [
    "spgemm_status_string", "spgemm_plan_workspace_size", "spgemm_plan_create", "spgemm_symbolic",
    "spgemm_numeric", "spgemm_numeric_static", "spgemm_numeric_static_limit", "spgemm_compute_only", "spgemm_plan_info", "spgemm_plan_last_hip_error", "spgemm_plan_destroy",
    "spgemm_model_create", "spgemm_model_get", "spgemm_model_save", "spgemm_model_load",
    "spgemm_model_destroy", "spgemm_model_device_bytes", "spgemm_model_upload", "spgemm_row_features",
    "spgemm_model_stats_scratch", "spgemm_model_feature_stats", "spgemm_model_grad_scratch",
    "spgemm_model_loss_grad", "spgemm_model_train_scratch", "spgemm_model_train", "spgemm_model_predict",
]

spgemm_batched_plan = _sig("spgemm_batched_plan", ctypes.c_int,
                           [I64, CSR_P, CSR_P, OPT_P, I64_P, SZ_P, ctypes.POINTER(P)])
spgemm_batched_reserve = _sig("spgemm_batched_reserve", ctypes.c_int, [P, P, SZ, I64_P, SZ_P, P])
spgemm_batched = _sig("spgemm_batched", ctypes.c_int, [P, P, SZ, P, P, P, I64, I64_P, I64_P, I64_P, P])
spgemm_batched_uses_graph = _sig("spgemm_batched_uses_graph", ctypes.c_int, [P])
spgemm_batched_destroy = _sig("spgemm_batched_destroy", None, [P])
EXPORTED += ["spgemm_batched_plan", "spgemm_batched_reserve", "spgemm_batched", "spgemm_batched_uses_graph",
             "spgemm_batched_destroy"]

spgemm_transpose_scratch = _sig("spgemm_transpose_scratch", SZ, [CSR_P])
spgemm_transpose = _sig("spgemm_transpose", ctypes.c_int, [CSR_P, P, P, P, P, SZ, P])
EXPORTED += ["spgemm_transpose_scratch", "spgemm_transpose"]


class SpgemmError(RuntimeError):
    def __init__(self, code: int, where: str, extra: str = ""):
        self.code = code
        super().__init__("%s failed: %s (%d)%s" % (where, STATUS.get(code, "?"), code, extra))


def check(code: int, where: str):
    if code != SPGEMM_OK:
        raise SpgemmError(code, where)
