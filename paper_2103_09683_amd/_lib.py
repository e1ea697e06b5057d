"""ctypes declarations of libdose's C ABI (include/dose.h).

Argument marshalling only: every computation happens in the HIP library.
Loading fails loudly when libdose.so has not been built; there is no
fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdose.so")

OK = 0
ERR_INVALID_ARGUMENT = -1
ERR_BAD_CSR = -2
ERR_UNSUPPORTED = -3
ERR_NO_TRANSPOSE = -4
ERR_OUT_OF_MEMORY = -5
ERR_HIP = -6
ERR_INTERNAL = -7

VAL_FP16, VAL_BF16, VAL_FP8E4M3_ROWSCALE, VAL_FP32 = 1, 2, 3, 4
IDX_I32 = 1
IDX_U16 = 2
IDX_RUNS = 3
CREATE_TRANSPOSE = 1
CREATE_AUTOTUNE = 2
CREATE_TRANSPOSE_SLABS = 4
ADJOINT_ACCUMULATE = 2
PART_A, PART_AT = 0, 1
PLAN_AUTOTUNE = 1
ROBUST_EXPECTED, ROBUST_WORST = 0, 1


class CsrHost(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col_idx", ctypes.c_void_p),
                ("values", ctypes.c_void_p)]


class MatrixInfo(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("value_format", ctypes.c_int32), ("index_format", ctypes.c_int32),
                ("has_transpose", ctypes.c_int32), ("group_nnz", ctypes.c_int32),
                ("n_groups", ctypes.c_int64), ("n_groups_windowed", ctypes.c_int64),
                ("group_nnz_t", ctypes.c_int32), ("slab_voxels", ctypes.c_int32),
                ("n_groups_t", ctypes.c_int64), ("n_groups_windowed_t", ctypes.c_int64),
                ("device_bytes", ctypes.c_uint64), ("spmv_bytes", ctypes.c_uint64),
                ("adjoint_bytes", ctypes.c_uint64), ("n_groups_split", ctypes.c_int64),
                ("n_groups_split_t", ctypes.c_int64)]


class BatchItem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("n_rhs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("ldy", ctypes.c_int64)]


class AdjointItem(ctypes.Structure):
    _fields_ = [("A", ctypes.c_void_p), ("reserved", ctypes.c_int32), ("v", ctypes.c_void_p),
                ("g", ctypes.c_void_p)]


class SellBatchItem(ctypes.Structure):
    _fields_ = [("S", ctypes.c_void_p), ("n_rhs", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("x", ctypes.c_void_p), ("ldx", ctypes.c_int64), ("y", ctypes.c_void_p),
                ("ldy", ctypes.c_int64)]


class SellInfo(ctypes.Structure):
    _fields_ = [("n_rows", ctypes.c_int64), ("n_cols", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("value_format", ctypes.c_int32), ("index_format", ctypes.c_int32),
                ("chunk_rows", ctypes.c_int32), ("sigma", ctypes.c_int32),
                ("n_chunks", ctypes.c_int64), ("n_groups", ctypes.c_int64),
                ("n_groups_windowed", ctypes.c_int64), ("std_slots", ctypes.c_int64),
                ("n_runs", ctypes.c_int64), ("stored_slots", ctypes.c_int64), ("device_bytes", ctypes.c_uint64),
                ("spmv_bytes", ctypes.c_uint64), ("stream_bytes", ctypes.c_uint64)]


# name -> (argtypes, restype); every entry point declared in include/dose.h
_vp, _i32, _i64, _u32, _u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                               ctypes.c_uint64)
SIGNATURES = {
    "dose_csr_validate": ([ctypes.POINTER(CsrHost), _i32, _i32], _i32),
    "dose_matrix_create": ([ctypes.POINTER(CsrHost), _i32, _i32, _u32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_matrix_set_partition": ([_vp, _i32, _i32], _i32),
    "dose_matrix_decode": ([_vp, _i32, _i64, _i64, _vp, _vp, _vp], _i32),
    "dose_matrix_info": ([_vp, ctypes.POINTER(MatrixInfo)], _i32),
    "dose_matrix_destroy": ([_vp], _i32),
    "dose_spmv": ([_vp, _vp, _vp, _vp], _i32),
    "dose_spmv_adjoint": ([_vp, _vp, _vp, _vp], _i32),
    "dose_spmv_f64": ([_vp, _vp, _vp, _vp], _i32),
    "dose_spmv_adjoint_f64": ([_vp, _vp, _vp, _vp], _i32),
    "dose_spmv_batched": ([ctypes.POINTER(BatchItem), _i32, _vp], _i32),
    "dose_batch_plan_create": ([ctypes.POINTER(BatchItem), _i32, _u32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_batch_plan_launch": ([_vp, _vp], _i32),
    "dose_adjoint_plan_create": ([ctypes.POINTER(AdjointItem), _i32, _u32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_scenario_plan_create": ([_vp, _vp, _i32, _i32, _vp, _u32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_batch_plan_destroy": ([_vp], _i32),
    "dose_objective": ([_i64, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "dose_norm2": ([_i64, _vp, _vp, _vp], _i32),
    "dose_robust_seed": ([_i32, _i64, _i32, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "dose_scenario_objective": ([_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "dose_scenario_objective_noalloc": ([_i32, _i32, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "dose_probe_stream_read": ([_vp, _u64, _vp, _vp], _i32),
    "dose_probe_copy": ([_vp, _vp, _u64, _vp], _i32),
    "dose_partition_preview": ([_vp, _i64, _i32, _vp, _i64, ctypes.POINTER(_i64)], _i32),
    "dose_sell_layout": ([_vp, _i64, _i32, _vp, _vp], _i32),
    "dose_sell_create": ([ctypes.POINTER(CsrHost), _i32, _i32, _i32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_sell_info": ([_vp, ctypes.POINTER(SellInfo)], _i32),
    "dose_sell_decode": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "dose_sell_runs": ([_vp, _vp, _vp, _vp], _i32),
    "dose_sell_spmv": ([_vp, _vp, _vp, _vp], _i32),
    "dose_sell_spmv_multi": ([_vp, _i32, _vp, _vp, _vp], _i32),
    "dose_sell_spmv_f64": ([_vp, _vp, _vp, _vp], _i32),
    "dose_sell_batch_plan_create": ([ctypes.POINTER(SellBatchItem), _i32, _u32, _vp, ctypes.POINTER(_vp)], _i32),
    "dose_sell_destroy": ([_vp], _i32),
    "dose_status_string": ([_i32], ctypes.c_char_p),
    "dose_last_error": ([], ctypes.c_char_p),
}

_lib = None


class DoseError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"{message} (status {code})")
        self.code = code
        self.message = message


def load():
    """The loaded library; raises if libdose.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run `python -m paper_2103_09683_amd.build` "
                               "(or __graft_entry__.build()) first")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(lib, name)
            f.argtypes = args
            f.restype = res
        _lib = lib
    return _lib


def check(status: int) -> None:
    if status != OK:
        lib = load()
        msg = lib.dose_last_error().decode(errors="replace")
        raise DoseError(status, msg or lib.dose_status_string(status).decode())
