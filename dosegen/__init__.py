"""Seeded synthetic inputs for the dose product d = A x.

The paper's six patient matrices (Table I) are not public, so every matrix
here is synthetic, shaped after the paper's description of dose-deposition
matrices (Sec. II-A, II-B): rows are voxels, columns are pencil-beam spots on
scanlines, most rows are empty, and a non-empty row holds a few contiguous
runs of spots around the voxel's beam's-eye-view position.

This module holds no part of the dose computation; it only produces the
arrays that both the CPU oracle and the GPU library consume.  The native part
(``dosegen.c``) is row-random-access: any row can be regenerated alone, which
lets the oracle check sampled rows of matrices too large to keep twice.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dosegen.c")
_LIB_PATH = os.path.join(_HERE, "libdosegen.so")
_lib = None


def build() -> str:
    """Compile libdosegen.so with gcc (OpenMP); returns its path."""
    tmp = _LIB_PATH + ".tmp"
    subprocess.check_call(["gcc", "-O2", "-fno-fast-math", "-fopenmp", "-fPIC", "-shared",
                           "-std=c11", "-Wall", "-o", tmp, _SRC, "-lm"])
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


class _Spec(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
                ("n_lines", ctypes.c_int32), ("n_spots", ctypes.c_int32),
                ("mean_len", ctypes.c_double), ("sigma_len", ctypes.c_double),
                ("max_len", ctypes.c_int32), ("beam_axis", ctypes.c_int32),
                ("empty_frac", ctypes.c_double), ("shift_u", ctypes.c_double),
                ("shift_v", ctypes.c_double), ("val_mu", ctypes.c_double),
                ("val_sigma", ctypes.c_double), ("seed", ctypes.c_uint64),
                ("matrix_id", ctypes.c_uint64)]


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            build()
        lib = ctypes.CDLL(_LIB_PATH)
        P = ctypes.POINTER(_Spec)
        i64, vp = ctypes.c_int64, ctypes.c_void_p
        lib.dg_row_len.argtypes = [P, i64]
        lib.dg_row_len.restype = i64
        lib.dg_row_lens.argtypes = [P, i64, i64, vp]
        lib.dg_row_lens.restype = None
        lib.dg_row.argtypes = [P, i64, vp, vp]
        lib.dg_row.restype = i64
        lib.dg_fill_rows.argtypes = [P, i64, i64, vp, vp, vp]
        lib.dg_fill_rows.restype = None
        lib.dg_fill_x.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, vp]
        lib.dg_fill_x.restype = None
        lib.dg_fill_signed.argtypes = [ctypes.c_uint64, ctypes.c_uint64, i64, vp]
        lib.dg_fill_signed.restype = None
        lib.dg_count_nonempty.argtypes = [P]
        lib.dg_count_nonempty.restype = i64
        lib.dg_num_threads.argtypes = []
        lib.dg_num_threads.restype = ctypes.c_int
        _lib = lib
    return _lib


def _ptr(a: np.ndarray) -> int:
    return a.ctypes.data


@dataclasses.dataclass(frozen=True)
class Spec:
    """One synthetic dose-deposition matrix.

    ``mean_nnz_per_row`` is averaged over ALL rows, empty ones included; the
    non-empty mean is derived from the realised footprint so that the total
    nnz lands on ``n_rows * mean_nnz_per_row`` up to sampling noise.
    """
    name: str
    nx: int
    ny: int
    nz: int
    n_lines: int
    n_spots: int
    mean_nnz_per_row: float
    empty_frac: float = 0.0
    sigma_len: float = 0.5
    max_len: int = 0
    beam_axis: int = 0
    shift_u: float = 0.0
    shift_v: float = 0.0
    val_mu: float = -3.0
    val_sigma: float = 1.0
    seed: int = 2103096830
    matrix_id: int = 0

    @property
    def n_rows(self) -> int:
        return self.nx * self.ny * self.nz

    @property
    def n_cols(self) -> int:
        return self.n_lines * self.n_spots

    def _c(self) -> _Spec:
        s = _Spec(self.nx, self.ny, self.nz, self.n_lines, self.n_spots, 1.0, self.sigma_len,
                  self.max_len, self.beam_axis, self.empty_frac, self.shift_u, self.shift_v,
                  self.val_mu, self.val_sigma, self.seed, self.matrix_id)
        n_ne = _load().dg_count_nonempty(ctypes.byref(s))
        s.mean_len = self.mean_nnz_per_row * self.n_rows / max(n_ne, 1)
        return s


def count_nonempty(spec: Spec) -> int:
    return int(_load().dg_count_nonempty(ctypes.byref(spec._c())))


def row_lens(spec: Spec, r0: int = 0, r1: int | None = None) -> np.ndarray:
    r1 = spec.n_rows if r1 is None else r1
    out = np.empty(r1 - r0, dtype=np.int32)
    _load().dg_row_lens(ctypes.byref(spec._c()), r0, r1, _ptr(out))
    return out


def row(spec: Spec, i: int) -> tuple[np.ndarray, np.ndarray]:
    """Columns (int32, strictly ascending) and FP32 values of row ``i``."""
    c = spec._c()
    n = _load().dg_row_len(ctypes.byref(c), i)
    cols = np.empty(max(n, 1), dtype=np.int32)
    vals = np.empty(max(n, 1), dtype=np.float32)
    _load().dg_row(ctypes.byref(c), i, _ptr(cols), _ptr(vals))
    return cols[:n], vals[:n]


def csr(spec: Spec, r0: int = 0, r1: int | None = None):
    """Rows [r0, r1) as host CSR: (row_ptr int64 starting at 0, cols int32, vals float32)."""
    r1 = spec.n_rows if r1 is None else r1
    c = spec._c()
    lens = np.empty(r1 - r0, dtype=np.int32)
    _load().dg_row_lens(ctypes.byref(c), r0, r1, _ptr(lens))
    row_ptr = np.zeros(r1 - r0 + 1, dtype=np.int64)
    np.cumsum(lens, out=row_ptr[1:])
    nnz = int(row_ptr[-1])
    cols = np.empty(max(nnz, 1), dtype=np.int32)
    vals = np.empty(max(nnz, 1), dtype=np.float32)
    _load().dg_fill_rows(ctypes.byref(c), r0, r1, _ptr(row_ptr), _ptr(cols), _ptr(vals))
    return row_ptr, cols[:nnz], vals[:nnz]


def spot_weights(seed: int, stream: int, n: int) -> np.ndarray:
    """x uniform in [0,1), each value (u32 >> 8) * 2^-24, exact in FP32."""
    x = np.empty(max(n, 1), dtype=np.float32)
    _load().dg_fill_x(seed, stream, n, _ptr(x))
    return x[:n]


def signed_values(seed: int, stream: int, n: int) -> np.ndarray:
    """Values k/128 for k in [-128, 128), exact in FP32."""
    x = np.empty(max(n, 1), dtype=np.float32)
    _load().dg_fill_signed(seed, stream, n, _ptr(x))
    return x[:n]


def num_threads() -> int:
    return int(_load().dg_num_threads())


# ---------------------------------------------------------------------------
# Workloads.  Seeds are 2103096830 + workload number.
# ---------------------------------------------------------------------------
SEED0 = 2103096830


def small_plain() -> Spec:
    """20,000 voxels (25x25x32) x 500 spots (20 lines x 25), ~40 nnz/row, no empty rows."""
    return Spec("small_plain_20000x500", 25, 25, 32, 20, 25, 40.0, 0.0, seed=SEED0 + 1)


def clinical_beam() -> Spec:
    """128^3 = 2,097,152 voxels x 25,000 spots (100 x 250), ~200 nnz/row over all rows, 60% empty."""
    return Spec("clinical_beam_2097152x25000", 128, 128, 128, 100, 250, 200.0, 0.6, seed=SEED0 + 2)


def sweep_large() -> Spec:
    """256x256x128 = 8,388,608 voxels x 60,000 spots (200 x 300), ~200 nnz/row, 60% empty."""
    return Spec("sweep_large_8388608x60000", 256, 256, 128, 200, 300, 200.0, 0.6, seed=SEED0 + 5)


def paper_irregular(base: Spec) -> Spec:
    """Heavier row-length tail (sigma 1.0, rows up to 16,000 nnz), as the paper reports for liver."""
    return dataclasses.replace(base, name=base.name + "_irregular", sigma_len=1.0, max_len=16000)


def beam_along_x(base: Spec) -> Spec:
    """Beam along x: neighbouring rows no longer share spots (no row-order locality of columns)."""
    return dataclasses.replace(base, name=base.name + "_beamx", beam_axis=1)


def robust_batch(scale: float = 1.0) -> list[Spec]:
    """9 setup-shift scenarios x 4 beams = 36 matrices of uneven sizes.

    Rows 0.5M-2.1M (128 x 128 x nz), spots 5k-25k (250 per scanline),
    50-250 nnz/row over all rows, 60% empty; scenario s shifts the footprint on
    a 3x3 pattern, beam b alternates the beam axis.  ``scale`` < 1 shrinks the
    grid depth (rows) for quick tests.
    """
    rng = np.random.default_rng(SEED0 + 3)
    specs = []
    for m in range(36):
        s, b = divmod(m, 4)
        nz = int(rng.integers(31, 129))
        n_lines = int(rng.integers(20, 101))
        mean = float(rng.uniform(50.0, 250.0))
        nz = max(2, int(round(nz * scale)))
        du = 0.02 * ((s % 3) - 1)
        dv = 0.02 * ((s // 3) - 1)
        specs.append(Spec(f"robust_s{s}_b{b}", 128, 128, nz, n_lines, 250, mean, 0.6,
                          beam_axis=b % 2, shift_u=du, shift_v=dv, seed=SEED0 + 3, matrix_id=m))
    return specs


def robust_scenarios(scale: float = 1.0, n_scen: int = 9, n_beams: int = 4, nx: int = 128, ny: int = 128,
                     spots_per_line: int = 250) -> list[Spec]:
    """n_scen setup-shift scenarios x n_beams beams on ONE shared dose grid,
    scenario-major (matrix s * n_beams + b is beam b under scenario s).

    Every beam of a scenario deposits into the same nx x ny x nz voxels
    (nz = 64 * scale), so a scenario's dose is the sum of its beams' doses.
    Beam b keeps its spots (20-100 scanlines of ``spots_per_line``) and its
    mean row length (50-250 over all rows, 60% empty) in every scenario;
    scenario s shifts the footprint on a 3x3 pattern and draws its own values;
    the beam axis alternates with b.
    """
    rng = np.random.default_rng(SEED0 + 6)
    nz = max(2, int(round(64 * scale)))
    beams = [(int(rng.integers(20, 101)), float(rng.uniform(50.0, 250.0))) for _ in range(n_beams)]
    specs = []
    for s in range(n_scen):
        du = 0.02 * ((s % 3) - 1)
        dv = 0.02 * (((s // 3) % 3) - 1)
        for b, (n_lines, mean) in enumerate(beams):
            specs.append(Spec(f"scenario_s{s}_b{b}", nx, ny, nz, n_lines, spots_per_line, mean, 0.6,
                              beam_axis=b % 2, shift_u=du, shift_v=dv, seed=SEED0 + 6,
                              matrix_id=s * n_beams + b))
    return specs


def objective_masks(nx: int = 25, ny: int = 25, nz: int = 32):
    """Prescription p and weights w on the dose grid (row = ix + nx*(iy + ny*iz)).

    Target: ball of radius 6 voxels at the grid centre, p = 60, w = 10.
    Organ at risk: the 5x5x6 box whose low-x face touches the ball's +x side,
    p = 20, w = 10.  Everything else: p = 0, w = 1.
    """
    iz, iy, ix = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
    cx, cy, cz = (nx - 1) / 2.0, (ny - 1) / 2.0, (nz - 1) / 2.0
    ball = (ix - cx) ** 2 + (iy - cy) ** 2 + (iz - cz) ** 2 <= 36.0
    x0 = int(np.floor(cx + 6.0)) + 1
    box = (ix >= x0) & (ix < x0 + 5) & (np.abs(iy - cy) <= 2.5) & (np.abs(iz - cz) <= 3.0)
    box &= ~ball
    p = np.zeros((nz, ny, nx), dtype=np.float32)
    w = np.ones((nz, ny, nx), dtype=np.float32)
    p[ball], w[ball] = 60.0, 10.0
    p[box], w[box] = 20.0, 10.0
    return p.reshape(-1), w.reshape(-1)
