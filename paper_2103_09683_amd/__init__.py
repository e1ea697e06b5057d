"""Dose product d = A x on MI355X (gfx950): Python binding of libdose.

The dose-deposition matrix A (voxels x spots, Sec. II-A/II-B of the paper)
is stored on the device in the paper's CSR format (FP16 values, int32
columns) or in BF16 / E4M3-with-row-scale variants; products accumulate in
FP32 and are bitwise reproducible (Sec. II-D).  This module only marshals
arguments to the C ABI in include/dose.h: PyTorch provides device memory and
streams, every step of the product runs in libdose's HIP kernels.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import DoseError

__all__ = ["DoseError", "DoseMatrix", "SellMatrix", "sell_layout", "BatchPlan", "SellBatchPlan", "ScenarioPlan", "spmv_batched", "objective", "norm2", "scenario_objective",
           "ScenarioObjective", "robust_seed",
           "csr_validate", "partition_preview", "byte_model", "DoseSpMV", "DoseObjective",
           "dose", "VALUE_FORMATS"]

VALUE_FORMATS = {"fp16": _lib.VAL_FP16, "bf16": _lib.VAL_BF16,
                 "fp8e4m3_rowscale": _lib.VAL_FP8E4M3_ROWSCALE, "fp32": _lib.VAL_FP32}
VALUE_BYTES = {"fp16": 2, "bf16": 2, "fp8e4m3_rowscale": 1, "fp32": 4}
INDEX_FORMATS = {"i32": _lib.IDX_I32, "u16": _lib.IDX_U16, "runs": _lib.IDX_RUNS}


def _stream_handle(stream) -> int | None:
    if stream is None:
        stream = torch.cuda.current_stream()
    return stream.cuda_stream


def _dev_ptr(t: torch.Tensor, n: int, name: str, device=None, dtype=torch.float32) -> int:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA tensor")
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be contiguous {str(dtype).replace('torch.', '')}")
    if t.numel() != n:
        raise ValueError(f"{name} has {t.numel()} elements, expected {n}")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, the matrix on {device}")
    return t.data_ptr()


def _csr_struct(row_ptr, cols, vals, n_cols):
    row_ptr = np.ascontiguousarray(row_ptr, dtype=np.int64)
    cols = np.ascontiguousarray(cols, dtype=np.int32)
    vals = np.ascontiguousarray(vals, dtype=np.float32)
    n_rows = row_ptr.size - 1
    c = _lib.CsrHost(n_rows, int(n_cols), int(cols.size), row_ptr.ctypes.data,
                     cols.ctypes.data if cols.size else None,
                     vals.ctypes.data if vals.size else None)
    return c, (row_ptr, cols, vals)


def csr_validate(row_ptr, cols, vals, n_cols, value_format: str = "fp16", index_format: str = "i32") -> int:
    """Host-only validation; returns the dose_status (0 = valid)."""
    c, keep = _csr_struct(row_ptr, cols, vals, n_cols)
    return int(_lib.load().dose_csr_validate(ctypes.byref(c), VALUE_FORMATS[value_format],
                                             INDEX_FORMATS[index_format]))


def partition_preview(row_ptr, group_nnz: int) -> np.ndarray:
    """Row groups the library builds for ``row_ptr`` (host only): one row per
    group, [r0, r1, r2, r3, r4, split].  The group holds rows [r0, r4); its
    wave w computes rows [r_w, r_(w+1)), unless ``split`` is 1: then the group
    is the single long row r0 and its four waves share that row's steps."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    lib = _lib.load()
    n = ctypes.c_int64(0)
    _lib.check(lib.dose_partition_preview(rp.ctypes.data, rp.size - 1, group_nnz, None, 0,
                                          ctypes.byref(n)))
    out = np.zeros((max(n.value, 1), 6), np.int64)
    _lib.check(lib.dose_partition_preview(rp.ctypes.data, rp.size - 1, group_nnz,
                                          out.ctypes.data, n.value, ctypes.byref(n)))
    return out[:n.value]


def byte_model(nnz, n_rows, n_cols, value_bytes=2, index_bytes=4, row_ptr_bytes=4,
               scale_bytes=0, x_bytes=4, y_bytes=4, n_rhs=1) -> float:
    """Algorithmic HBM bytes of one product with an ideal cache (Sec. V):
    every stored entry, every row offset (one per row) and every row scale is
    read once, x is read once and y written once.  With FP16 values, int32
    indices and FP64 x/y this is the paper's 6 nnz + 12 nr + 8 nc."""
    return (nnz * (value_bytes + index_bytes) + n_rows * (row_ptr_bytes + scale_bytes)
            + n_rhs * (n_cols * x_bytes + n_rows * y_bytes))


def storage_bytes(nnz, n_rows, value_bytes=2, index_bytes=4, row_ptr_bytes=4) -> float:
    """Bytes of a CSR matrix: values, column indices and n_rows+1 row offsets."""
    return nnz * (value_bytes + index_bytes) + (n_rows + 1) * row_ptr_bytes


class DoseMatrix:
    """A dose-deposition matrix on the current HIP device.

    row_ptr (int64, n_rows+1), cols (int32) and vals (float32) are host CSR
    arrays; they are validated, uploaded and encoded once.  With
    ``transpose=True`` A^T is stored as well for :meth:`adjoint`
    (``transpose="slabs"``: in voxel slabs, whose adjoint reads the seed from
    LDS and adds each spot's slab partials in a fixed order); with
    ``autotune=True`` the row-group sizes of the plain products are chosen by
    timing them (speed only: results are bitwise the same).
    """

    def __init__(self, row_ptr, cols, vals, n_cols: int, value_format: str = "fp16",
                 transpose: bool | str = False, stream=None, index_format: str = "i32", autotune: bool = False):
        slabs = isinstance(transpose, str)
        if slabs and transpose != "slabs":
            raise ValueError(f"transpose must be a bool or 'slabs', not {transpose!r}")
        if value_format not in VALUE_FORMATS:
            raise ValueError(f"unknown value format {value_format!r}")
        if index_format not in INDEX_FORMATS:
            raise ValueError(f"unknown index format {index_format!r}")
        self._h = None
        lib = _lib.load()
        c, keep = _csr_struct(row_ptr, cols, vals, n_cols)
        h = ctypes.c_void_p()
        _lib.check(lib.dose_matrix_create(ctypes.byref(c), VALUE_FORMATS[value_format],
                                          INDEX_FORMATS[index_format],
                                          (_lib.CREATE_TRANSPOSE if transpose and not slabs else 0) |
                                          (_lib.CREATE_TRANSPOSE_SLABS if slabs else 0) |
                                          (_lib.CREATE_AUTOTUNE if autotune else 0),
                                          _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.value_format = value_format
        self.index_format = index_format
        self.n_rows = int(c.n_rows)
        self.n_cols = int(c.n_cols)
        self.nnz = int(c.nnz)
        self.has_transpose = bool(transpose)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @property
    def handle(self) -> int:
        if self._h is None:
            raise RuntimeError("matrix is closed")
        return self._h.value

    def info(self) -> dict:
        inf = _lib.MatrixInfo()
        _lib.check(_lib.load().dose_matrix_info(self.handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _lib.MatrixInfo._fields_}

    def set_partition(self, group_nnz: int, group_nnz_t: int | None = None) -> None:
        """Row groups of about ``group_nnz`` entries (speed only: results are
        bitwise the same under any partition)."""
        gt = group_nnz_t if group_nnz_t is not None else (self.info()["group_nnz_t"] or group_nnz)
        _lib.check(_lib.load().dose_matrix_set_partition(self.handle, group_nnz, gt))

    def decode(self, row_begin: int = 0, row_end: int | None = None, part: str = "A"):
        """Host CSR of rows [row_begin, row_end) decoded to FP32 on the device."""
        p = _lib.PART_A if part == "A" else _lib.PART_AT
        n_rows = self.n_rows if p == _lib.PART_A else self.n_cols
        row_end = n_rows if row_end is None else row_end
        lib = _lib.load()
        rp = np.zeros(max(row_end - row_begin, 0) + 1, np.int64)
        _lib.check(lib.dose_matrix_decode(self.handle, p, row_begin, row_end, rp.ctypes.data,
                                          None, None))
        n = int(rp[-1])
        cols = np.empty(max(n, 1), np.int32)
        vals = np.empty(max(n, 1), np.float32)
        _lib.check(lib.dose_matrix_decode(self.handle, p, row_begin, row_end, rp.ctypes.data,
                                          cols.ctypes.data, vals.ctypes.data))
        return rp, cols[:n], vals[:n]

    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """y = A x, asynchronous on the current (or given) stream.  FP32 x
        gives FP32 y; FP64 x gives FP64 y with FP64 products and sums (the
        paper's half/double configuration)."""
        f64 = x.dtype == torch.float64
        dt = torch.float64 if f64 else torch.float32
        if y is None:
            y = torch.empty(self.n_rows, dtype=dt, device=x.device)
        fn = _lib.load().dose_spmv_f64 if f64 else _lib.load().dose_spmv
        _lib.check(fn(self.handle, _dev_ptr(x, self.n_cols, "x", self.device, dt),
                      _dev_ptr(y, self.n_rows, "y", self.device, dt), _stream_handle(stream)))
        return y

    def adjoint(self, v: torch.Tensor, g: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """g = A^T v, asynchronous; FP64 v gives FP64 g as for spmv."""
        f64 = v.dtype == torch.float64
        dt = torch.float64 if f64 else torch.float32
        if g is None:
            g = torch.empty(self.n_cols, dtype=dt, device=v.device)
        fn = _lib.load().dose_spmv_adjoint_f64 if f64 else _lib.load().dose_spmv_adjoint
        _lib.check(fn(self.handle, _dev_ptr(v, self.n_rows, "v", self.device, dt),
                      _dev_ptr(g, self.n_cols, "g", self.device, dt), _stream_handle(stream)))
        return g

    def close(self) -> None:
        if self._h is not None:
            _lib.check(_lib.load().dose_matrix_destroy(self._h.value))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def sell_layout(row_ptr, sigma: int):
    """SELL-C-sigma layout the library builds (host only, C = 64): (perm,
    width), perm[k] the row at sorted position k, width[c] the longest row of
    chunk c."""
    rp = np.ascontiguousarray(row_ptr, dtype=np.int64)
    n = rp.size - 1
    perm = np.empty(max(n, 1), np.int64)
    width = np.empty(max((n + 63) // 64, 1), np.int64)
    _lib.check(_lib.load().dose_sell_layout(rp.ctypes.data, n, int(sigma), perm.ctypes.data, width.ctypes.data))
    return perm[:n], width[:(n + 63) // 64]


class SellMatrix:
    """A dose-deposition matrix in SELL-C-sigma storage (C = 64) on the
    current HIP device: the same host CSR arrays and value/index formats as
    :class:`DoseMatrix`, rows sorted by length inside windows of ``sigma``."""

    def __init__(self, row_ptr, cols, vals, n_cols: int, value_format: str = "fp16", sigma: int = 65536,
                 index_format: str = "i32", stream=None):
        if value_format not in VALUE_FORMATS:
            raise ValueError(f"unknown value format {value_format!r}")
        if index_format not in INDEX_FORMATS:
            raise ValueError(f"unknown index format {index_format!r}")
        self._h = None
        c, keep = _csr_struct(row_ptr, cols, vals, n_cols)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().dose_sell_create(ctypes.byref(c), VALUE_FORMATS[value_format],
                                                INDEX_FORMATS[index_format], int(sigma),
                                                _stream_handle(stream), ctypes.byref(h)))
        self._h = h
        self.value_format = value_format
        self.index_format = index_format
        self.sigma = int(sigma)
        self.n_rows = int(c.n_rows)
        self.n_cols = int(c.n_cols)
        self.nnz = int(c.nnz)
        self.device = torch.device("cuda", torch.cuda.current_device())

    @property
    def handle(self) -> int:
        if self._h is None:
            raise RuntimeError("matrix is closed")
        return self._h.value

    def info(self) -> dict:
        inf = _lib.SellInfo()
        _lib.check(_lib.load().dose_sell_info(self.handle, ctypes.byref(inf)))
        return {name: getattr(inf, name) for name, _ in _lib.SellInfo._fields_}

    def decode(self):
        """(perm, width, val, col) in Kreutzer's column-major layout, values
        decoded to FP32; padding slots hold 0 and column -1."""
        inf = self.info()
        perm = np.empty(max(self.n_rows, 1), np.int64)
        width = np.empty(max(inf["n_chunks"], 1), np.int64)
        val = np.empty(max(inf["std_slots"], 1), np.float32)
        col = np.empty(max(inf["std_slots"], 1), np.int32)
        _lib.check(_lib.load().dose_sell_decode(self.handle, perm.ctypes.data, width.ctypes.data,
                                                val.ctypes.data, col.ctypes.data))
        n = inf["std_slots"]
        return perm[:self.n_rows], width[:inf["n_chunks"]], val[:n], col[:n]

    def runs(self):
        """Run-length indices (index format "runs") read back from the device,
        by row: (run_ptr, start, length)."""
        inf = self.info()
        run_ptr = np.empty(self.n_rows + 1, np.int64)
        start = np.empty(max(inf["n_runs"], 1), np.int32)
        length = np.empty(max(inf["n_runs"], 1), np.int32)
        _lib.check(_lib.load().dose_sell_runs(self.handle, run_ptr.ctypes.data, start.ctypes.data,
                                              length.ctypes.data))
        return run_ptr, start[:inf["n_runs"]], length[:inf["n_runs"]]

    def spmv(self, x: torch.Tensor, y: torch.Tensor | None = None, stream=None) -> torch.Tensor:
        """y = A x, asynchronous on the current (or given) stream.  FP32 x of
        shape (n_cols,) gives y (n_rows,); x (n_cols, n_rhs) with n_rhs 1, 2
        or 4 gives y (n_rows, n_rhs), each column bitwise the product of x's
        column; FP64 x (n_cols,) gives FP64 y with FP64 products and sums
        (the paper's half/double configuration)."""
        if x.dtype == torch.float64:
            if y is None:
                y = torch.empty(self.n_rows, dtype=torch.float64, device=x.device)
            _lib.check(_lib.load().dose_sell_spmv_f64(
                self.handle, _dev_ptr(x, self.n_cols, "x", self.device, torch.float64),
                _dev_ptr(y, self.n_rows, "y", self.device, torch.float64), _stream_handle(stream)))
            return y
        if x.dim() == 2:
            n_rhs = x.shape[1]
            if x.shape[0] != self.n_cols:
                raise ValueError(f"x has shape {tuple(x.shape)}, expected ({self.n_cols}, n_rhs)")
            if y is None:
                y = torch.empty(self.n_rows, n_rhs, dtype=torch.float32, device=x.device)
            if y.shape != (self.n_rows, n_rhs):
                raise ValueError(f"y has shape {tuple(y.shape)}, expected ({self.n_rows}, {n_rhs})")
            _lib.check(_lib.load().dose_sell_spmv_multi(
                self.handle, n_rhs, _dev_ptr(x, self.n_cols * n_rhs, "x", self.device),
                _dev_ptr(y, self.n_rows * n_rhs, "y", self.device), _stream_handle(stream)))
            return y
        if y is None:
            y = torch.empty(self.n_rows, dtype=torch.float32, device=x.device)
        _lib.check(_lib.load().dose_sell_spmv(self.handle, _dev_ptr(x, self.n_cols, "x", self.device),
                                              _dev_ptr(y, self.n_rows, "y", self.device), _stream_handle(stream)))
        return y

    def close(self) -> None:
        if self._h is not None:
            _lib.check(_lib.load().dose_sell_destroy(self._h.value))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _items(entries):
    """Batch items of (DoseMatrix, x, y) triples: x is (n_cols,) or
    (n_cols, n_rhs) and y (n_rows,) or (n_rows, n_rhs), both contiguous FP32
    on the matrix's device (the kernels read x as [n_cols][n_rhs])."""
    arr = (_lib.BatchItem * len(entries))()
    for i, (A, x, y) in enumerate(entries):
        for name, t in (("x", x), ("y", y)):
            if not isinstance(t, torch.Tensor) or t.dim() not in (1, 2):
                raise TypeError(f"item {i}: {name} must be a 1- or 2-dimensional tensor")
        n_rhs = 1 if x.dim() == 1 else x.shape[1]
        if x.shape != ((A.n_cols,) if x.dim() == 1 else (A.n_cols, n_rhs)):
            raise ValueError(f"item {i}: x has shape {tuple(x.shape)}, expected ({A.n_cols}[, n_rhs])")
        if y.shape != ((A.n_rows,) if x.dim() == 1 else (A.n_rows, n_rhs)):
            raise ValueError(f"item {i}: y has shape {tuple(y.shape)}, expected the rows of x's layout")
        _dev_ptr(x, A.n_cols * n_rhs, "x", A.device)
        _dev_ptr(y, A.n_rows * n_rhs, "y", A.device)
        arr[i] = _lib.BatchItem(A.handle, n_rhs, 0, x.data_ptr(), n_rhs, y.data_ptr(), n_rhs)
    return arr


def spmv_batched(entries, stream=None) -> None:
    """entries: list of (DoseMatrix, x [n_cols] or [n_cols, n_rhs], y [n_rows(, n_rhs)])."""
    arr = _items(entries)
    _lib.check(_lib.load().dose_spmv_batched(arr, len(entries), _stream_handle(stream)))


class BatchPlan:
    """A batched product captured once into a HIP graph and replayed."""

    def __init__(self, entries, autotune: bool = False, stream=None):
        self._h = None
        self._keep = list(entries)
        arr = _items(entries)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().dose_batch_plan_create(arr, len(entries),
                                                      _lib.PLAN_AUTOTUNE if autotune else 0,
                                                      _stream_handle(stream), ctypes.byref(h)))
        self._h = h

    def launch(self, stream=None) -> None:
        _lib.check(_lib.load().dose_batch_plan_launch(self._h.value, _stream_handle(stream)))

    def close(self) -> None:
        if self._h is not None:
            _lib.check(_lib.load().dose_batch_plan_destroy(self._h.value))
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class AdjointPlan(BatchPlan):
    """The adjoints g = A^T v of several matrices (each created with a
    transpose, all of one layout and value format) captured into one HIP
    graph and replayed by :meth:`launch`: entries are (DoseMatrix, v, g) with
    v (n_rows,) and g (n_cols,) contiguous FP32 on the matrix's device; each
    g gets the bits of ``A.adjoint(v)``.  ``autotune=True`` times the launch
    under candidate row-group sizes first (speed only).  ``accumulate=True``
    (matrices with A^T in voxel slabs): entries sharing the same g tensor sum
    their adjoints into it, in one fixed order (entry by entry, each in
    ascending slab)."""

    def __init__(self, entries, autotune: bool = False, accumulate: bool = False, stream=None):
        self._h = None
        self._keep = list(entries)
        arr = (_lib.AdjointItem * len(entries))()
        for i, (A, v, g) in enumerate(entries):
            _dev_ptr(v, A.n_rows, "v", A.device)
            _dev_ptr(g, A.n_cols, "g", A.device)
            arr[i] = _lib.AdjointItem(A.handle, 0, v.data_ptr(), g.data_ptr())
        h = ctypes.c_void_p()
        flags = (_lib.PLAN_AUTOTUNE if autotune else 0) | (_lib.ADJOINT_ACCUMULATE if accumulate else 0)
        _lib.check(_lib.load().dose_adjoint_plan_create(arr, len(entries), flags, _stream_handle(stream),
                                                        ctypes.byref(h)))
        self._h = h


class SellBatchPlan(BatchPlan):
    """Many SELL-C-sigma products in one launch, captured into a HIP graph:
    entries are (SellMatrix, x, y) with x (n_cols,) or (n_cols, n_rhs) and y
    (n_rows,) or (n_rows, n_rhs), contiguous FP32 on the matrix's device."""

    def __init__(self, entries, stream=None):
        self._h = None
        self._keep = list(entries)
        arr = (_lib.SellBatchItem * len(entries))()
        for i, (S, x, y) in enumerate(entries):
            for name, t in (("x", x), ("y", y)):
                if not isinstance(t, torch.Tensor) or t.dim() not in (1, 2):
                    raise TypeError(f"item {i}: {name} must be a 1- or 2-dimensional tensor")
            n_rhs = 1 if x.dim() == 1 else x.shape[1]
            if x.shape != ((S.n_cols,) if x.dim() == 1 else (S.n_cols, n_rhs)):
                raise ValueError(f"item {i}: x has shape {tuple(x.shape)}, expected ({S.n_cols}[, n_rhs])")
            if y.shape != ((S.n_rows,) if x.dim() == 1 else (S.n_rows, n_rhs)):
                raise ValueError(f"item {i}: y has shape {tuple(y.shape)}, expected the rows of x's layout")
            _dev_ptr(x, S.n_cols * n_rhs, "x", S.device)
            _dev_ptr(y, S.n_rows * n_rhs, "y", S.device)
            arr[i] = _lib.SellBatchItem(S.handle, n_rhs, 0, x.data_ptr(), n_rhs, y.data_ptr(), n_rhs)
        h = ctypes.c_void_p()
        _lib.check(_lib.load().dose_sell_batch_plan_create(arr, len(entries), 0, _stream_handle(stream),
                                                           ctypes.byref(h)))
        self._h = h


class ScenarioPlan(BatchPlan):
    """Scenario doses of a robust plan in one graph launch: ``d[s] = sum_b
    A[s][b] x[s][b]`` (FP32, ascending beam order, the beam sum done by the
    products: one launch per beam, the first storing, the others adding).
    ``mats`` and ``xs`` are n_scen x n_beams nested lists (DoseMatrix, FP32
    spot-weight tensors); ``d`` is (n_scen, n_rows) FP32."""

    def __init__(self, mats, xs, d: torch.Tensor, autotune: bool = False, stream=None):
        self._h = None
        n_scen, n_beams = len(mats), len(mats[0])
        if len(xs) != n_scen or any(len(row) != n_beams for row in mats) or any(len(row) != n_beams for row in xs):
            raise ValueError("mats and xs must be n_scen x n_beams")
        flat = [mats[s][b] for s in range(n_scen) for b in range(n_beams)]
        fx = [xs[s][b] for s in range(n_scen) for b in range(n_beams)]
        n = flat[0].n_rows
        if d.shape != (n_scen, n):
            raise ValueError(f"d has shape {tuple(d.shape)}, expected ({n_scen}, {n})")
        _dev_ptr(d, n_scen * n, "d", flat[0].device)
        for A, x in zip(flat, fx):
            _dev_ptr(x, A.n_cols, "x", A.device)
        self._keep = (flat, fx, d)
        ha = (ctypes.c_void_p * len(flat))(*[A.handle for A in flat])
        hx = (ctypes.c_void_p * len(fx))(*[x.data_ptr() for x in fx])
        h = ctypes.c_void_p()
        _lib.check(_lib.load().dose_scenario_plan_create(ha, hx, n_scen, n_beams, d.data_ptr(),
                                                         _lib.PLAN_AUTOTUNE if autotune else 0,
                                                         _stream_handle(stream), ctypes.byref(h)))
        self._h = h


def objective(d, p, w, seed: torch.Tensor | None = None, out: torch.Tensor | None = None,
              stream=None) -> torch.Tensor:
    """f = sum w (d - p)^2 in FP64 on the device (one-element float64 tensor);
    writes the FP32 adjoint seed 2 w (d - p) into ``seed`` if given."""
    n = d.numel()
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=d.device)
    _lib.check(_lib.load().dose_objective(
        n, _dev_ptr(d, n, "d"), _dev_ptr(p, n, "p"), _dev_ptr(w, n, "w"),
        _dev_ptr(seed, n, "seed") if seed is not None else None, out.data_ptr(),
        _stream_handle(stream)))
    return out


def scenario_objective(part: torch.Tensor, p, w, prob: torch.Tensor | None = None,
                       d_out: torch.Tensor | None = None, seed: torch.Tensor | None = None,
                       out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Robust epilogue over the beam doses ``part`` (n_scen, n_beams, n), FP32.

    Returns a float64 tensor of n_scen + 3 values on the device: the scenario
    objectives f_s = sum w (d_s - p)^2 with d_s the FP32 sum of the
    scenario's beam doses in ascending beam order, then max_s f_s, the
    expectation sum_s prob_s f_s (uniform without ``prob``) and the index of
    the first worst scenario.  Writes d_s into ``d_out`` (n_scen, n) and the
    FP32 seeds 2 w (d_s - p) into ``seed`` (n_scen, n) if given."""
    if part.dim() != 3:
        raise ValueError("part must be (n_scen, n_beams, n)")
    n_scen, n_beams, n = part.shape
    if out is None:
        out = torch.empty(n_scen + 3, dtype=torch.float64, device=part.device)
    _lib.check(_lib.load().dose_scenario_objective(
        n_scen, n_beams, n, _dev_ptr(part, part.numel(), "part"), _dev_ptr(p, n, "p"), _dev_ptr(w, n, "w"),
        _dev_ptr(prob, n_scen, "prob", dtype=torch.float64) if prob is not None else None,
        _dev_ptr(d_out, n_scen * n, "d_out") if d_out is not None else None,
        _dev_ptr(seed, n_scen * n, "seed") if seed is not None else None,
        _dev_ptr(out, n_scen + 3, "out", dtype=torch.float64), _stream_handle(stream)))
    return out


def robust_seed(seed: torch.Tensor, mode: str = "expected", out: torch.Tensor | None = None,
                prob: torch.Tensor | None = None, grad_scale: torch.Tensor | None = None,
                wseed: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """Seeds of the robust objective's gradient, (n_scen, n) FP32: scenario s's
    seed times c_s g, with c_s = prob_s (uniform without ``prob``) for mode
    "expected", or 1 for the first worst scenario (index read from ``out`` of
    :func:`scenario_objective`) and 0 for the others for mode "worst"; g is
    the one-element FP64 tensor ``grad_scale`` (1 without it)."""
    if mode not in ("expected", "worst"):
        raise ValueError("mode is 'expected' or 'worst'")
    if seed.dim() != 2:
        raise ValueError("seed must be (n_scen, n)")
    n_scen, n = seed.shape
    if wseed is None:
        wseed = torch.empty_like(seed)
    _lib.check(_lib.load().dose_robust_seed(
        n_scen, n, _lib.ROBUST_WORST if mode == "worst" else _lib.ROBUST_EXPECTED,
        _dev_ptr(out, n_scen + 3, "out", dtype=torch.float64) if out is not None else None,
        _dev_ptr(prob, n_scen, "prob", dtype=torch.float64) if prob is not None else None,
        _dev_ptr(grad_scale, 1, "grad_scale", dtype=torch.float64) if grad_scale is not None else None,
        _dev_ptr(seed, n_scen * n, "seed"), _dev_ptr(wseed, n_scen * n, "wseed"), _stream_handle(stream)))
    return wseed


def norm2(g: torch.Tensor, out: torch.Tensor | None = None, stream=None) -> torch.Tensor:
    """sqrt(sum g^2) in FP64 on the device."""
    if out is None:
        out = torch.empty(1, dtype=torch.float64, device=g.device)
    _lib.check(_lib.load().dose_norm2(g.numel(), _dev_ptr(g, g.numel(), "g"), out.data_ptr(),
                                      _stream_handle(stream)))
    return out


def probe_stream_read(buf: torch.Tensor, sink: torch.Tensor, stream=None) -> None:
    _lib.check(_lib.load().dose_probe_stream_read(buf.data_ptr(), buf.numel() * buf.element_size(),
                                                  sink.data_ptr(), _stream_handle(stream)))


def probe_copy(src: torch.Tensor, dst: torch.Tensor, stream=None) -> None:
    _lib.check(_lib.load().dose_probe_copy(src.data_ptr(), dst.data_ptr(),
                                           src.numel() * src.element_size(),
                                           _stream_handle(stream)))


class DoseSpMV(torch.autograd.Function):
    """d = A x with dL/dx = A^T dL/dd (the matrix needs transpose=True for
    backward).  FP32 x runs the FP32 products; FP64 x the FP64 ones (the
    paper's half/double configuration), forward and backward."""

    @staticmethod
    def forward(ctx, x, A):
        ctx.A = A
        ctx.f64 = x.dtype == torch.float64
        return A.spmv(x.contiguous())

    @staticmethod
    def backward(ctx, gd):
        gd = gd.contiguous().to(torch.float64 if ctx.f64 else torch.float32)
        return ctx.A.adjoint(gd), None


class DoseObjective(torch.autograd.Function):
    """f = sum w (d - p)^2 (FP64 reduction) with df/dd = 2 w (d - p)."""

    @staticmethod
    def forward(ctx, d, p, w):
        seed = torch.empty_like(d)
        f = objective(d.contiguous(), p.contiguous(), w.contiguous(), seed=seed)
        ctx.save_for_backward(seed)
        return f.reshape(())

    @staticmethod
    def backward(ctx, gf):
        (seed,) = ctx.saved_tensors
        # one scenario's expectation: the seed times the outer derivative
        g = robust_seed(seed.view(1, -1), "expected", grad_scale=gf.to(torch.float64).reshape(1).contiguous())
        return g.view(-1), None, None


class RobustProblem:
    """One robust plan-optimisation iteration in library calls (Sec. I, II-A):
    the dose of every beam under every scenario (one batch plan), the robust
    objective and the scenario seeds (FP64 reductions), the robust seeds, and
    each beam's gradient summed over the scenarios (one accumulating adjoint
    plan).  ``mats[s][b]`` is beam b's DoseMatrix under scenario s, all with
    A^T in voxel slabs, one voxel grid; ``xs[b]`` beam b's FP32 spot weights
    (read at every step: update them in place); ``p``, ``w`` the voxel
    prescription and weights; ``mode`` "expected" (with ``prob``, or uniform)
    or "worst".  :meth:`step` returns the n_scen + 3 FP64 values of
    :func:`scenario_objective` and the list of beam gradients (FP32, each
    ``(n_cols_b,)``), all on the device, asynchronously: they are the
    problem's own tensors, overwritten by the next step (clone to keep)."""

    def __init__(self, mats, xs, p: torch.Tensor, w: torch.Tensor, prob: torch.Tensor | None = None,
                 mode: str = "expected"):
        if mode not in ("expected", "worst"):
            raise ValueError("mode is 'expected' or 'worst'")
        n_scen, n_beams = len(mats), len(xs)
        if n_scen == 0 or any(len(row) != n_beams for row in mats):
            raise ValueError("mats must be n_scen lists of one matrix per beam")
        n = mats[0][0].n_rows
        if any(A.n_rows != n for row in mats for A in row):
            raise ValueError("every matrix must have the voxel grid's rows")
        for b in range(n_beams):
            if any(mats[s][b].n_cols != xs[b].numel() for s in range(n_scen)):
                raise ValueError(f"beam {b}: every scenario's matrix must have the beam's spots")
        dev = xs[0].device
        self.mats, self.xs, self.p, self.w, self.prob, self.mode = mats, xs, p, w, prob, mode
        self.part = torch.empty(n_scen, n_beams, n, dtype=torch.float32, device=dev)
        self.seed = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
        self.wseed = torch.empty(n_scen, n, dtype=torch.float32, device=dev)
        self.out = torch.empty(n_scen + 3, dtype=torch.float64, device=dev)
        self.grads = [torch.empty(x.numel(), dtype=torch.float32, device=dev) for x in xs]
        self._doses = BatchPlan([(mats[s][b], xs[b], self.part[s, b]) for s in range(n_scen) for b in range(n_beams)])
        self._adjoints = AdjointPlan([(mats[s][b], self.wseed[s], self.grads[b])
                                      for s in range(n_scen) for b in range(n_beams)], accumulate=True)

    def step(self, stream=None):
        self._doses.launch(stream)
        scenario_objective(self.part, self.p, self.w, prob=self.prob, seed=self.seed, out=self.out, stream=stream)
        robust_seed(self.seed, self.mode, out=self.out, prob=self.prob, wseed=self.wseed, stream=stream)
        self._adjoints.launch(stream)
        return self.out, self.grads

    def close(self) -> None:
        self._doses.close()
        self._adjoints.close()


class ScenarioObjective(torch.autograd.Function):
    """Robust objective of the beam doses part (n_scen, n_beams, n): the
    expectation sum_s prob_s f_s (mode "expected"; the mean without prob) or
    the worst case max_s f_s (mode "worst"), f_s = sum w (d_s - p)^2 with d_s
    the scenario's beam sum.  d/dpart[s, b] = c_s 2 w (d_s - p) for every beam
    b, with c_s = prob_s (expected) or 1 for the first worst scenario and 0
    otherwise (worst); the library forms these seeds (dose_robust_seed)."""

    @staticmethod
    def forward(ctx, part, p, w, prob=None, mode: str = "expected"):
        if mode not in ("expected", "worst"):
            raise ValueError("mode is 'expected' or 'worst'")
        part = part.contiguous()
        n_scen, n_beams, n = part.shape
        seed = torch.empty(n_scen, n, dtype=torch.float32, device=part.device)
        prob = None if prob is None else prob.contiguous()
        out = scenario_objective(part, p.contiguous(), w.contiguous(), prob=prob, seed=seed)
        ctx.save_for_backward(seed, out, prob)
        ctx.n_beams = n_beams
        ctx.mode = mode
        return out[n_scen + 1] if mode == "expected" else out[n_scen]

    @staticmethod
    def backward(ctx, gf):
        seed, out, prob = ctx.saved_tensors
        g = robust_seed(seed, ctx.mode, out=out, prob=prob,
                        grad_scale=gf.to(torch.float64).reshape(1).contiguous())
        return g[:, None, :].expand(-1, ctx.n_beams, -1), None, None, None, None


def dose(x: torch.Tensor, A: DoseMatrix) -> torch.Tensor:
    """Differentiable d = A x."""
    return DoseSpMV.apply(x, A)
